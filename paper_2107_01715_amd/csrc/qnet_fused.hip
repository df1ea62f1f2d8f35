// Fused convolution stack of the Nature-DQN (conv1 -> conv2 -> conv3) for
// BF16 / FP8 operands on the CDNA4 matrix cores, one workgroup per sibling
// group of eval items.
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
// Data path of a workgroup (4 wavefronts):
//   * a frame is read from HBM once, converted to the operand type once and
//     staged in LDS (double-buffered; the next item's frame is loaded into
//     registers while the current one is used);
//   * conv1 -> x1 (20x20x32) and conv2 -> x2 (9x9x64) of T items at a time
//     stay in LDS, in swizzled layouts that keep the MFMA operand reads free
//     of bank conflicts without padding;
//   * conv3 -> x3 (7x7x64, channels-last) goes to HBM for fc1.
// Every layer is an implicit GEMM computed transposed, D[channel][pixel] =
// W[channel][k] * X[k][pixel], with 16x16x32 MFMAs (BF16 or OCP e4m3, FP32
// accumulate): the weights are the A operand and the im2col pixels the B
// operand, so each lane ends with 4 consecutive channels of one pixel and
// stores them with one 8-byte (BF16) or 4-byte (FP8) write.  A wavefront owns
// a set of 16-pixel fragments and all channel fragments of a layer.  The sum
// order of every output element is fixed by the layer, never by the group
// size, round size or chunking, so results do not depend on batching.
#include "bcts_internal.h"

namespace bcts {
namespace {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

constexpr int kThreads = 256;
constexpr int kWaves = 4;
constexpr int kF1 = 7;                 // conv1 pixel fragments per wave: w, w+4, ... < 25

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
};

// Swizzled LDS layouts (byte offsets).  x1: per item 400 pixels x 32
// channels; two pixels form a row of 8 units and unit ((p&1)*4 + c/8) is
// stored at slot ^ ((p>>1) & 7).  x2: per item 81 pixels x 64 channels; one
// pixel is a row of 8 units, unit c/8 at slot ^ (p & 7).
template <int P> __device__ __forceinline__ int x1_off(int t, int p, int c) {
  constexpr int UB = F<P>::UB, EB = F<P>::EB;
  return t * 400 * 32 * EB + (p >> 1) * 8 * UB + (((((p & 1) << 2) | (c >> 3)) ^ ((p >> 1) & 7)) * UB) +
         (c & 7) * EB;
}
template <int P> __device__ __forceinline__ int x2_off(int t, int p, int c) {
  constexpr int UB = F<P>::UB, EB = F<P>::EB;
  return t * 81 * 64 * EB + p * 8 * UB + (((c >> 3) ^ (p & 7)) * UB) + (c & 7) * EB;
}

template <int P, int T>
__global__ void __launch_bounds__(kThreads, (T <= 2 ? 2 : 1)) conv_fused_kernel(FusedConvArgs a) {
  typedef F<P> Fr;
  typedef typename Fr::V V;
  constexpr int EB = Fr::EB;
  constexpr int FRB = kFrameBytes * EB;                 // staged frame bytes
  constexpr int R2 = T * 81, F2 = (R2 + 15) / 16, F2W = (F2 + kWaves - 1) / kWaves;
  constexpr int R3 = T * 49, F3 = (R3 + 15) / 16, F3W = (F3 + kWaves - 1) / kWaves;
  __shared__ __attribute__((aligned(16))) unsigned char x1[T * 400 * 32 * EB];
  __shared__ __attribute__((aligned(16))) unsigned char x2[T * 81 * 64 * EB];
  __shared__ __attribute__((aligned(16))) unsigned char fs[2][FRB];

  const FusedGroup grp = a.groups[blockIdx.x];
  const int G = grp.count;
  const long long i0 = grp.item0 - a.item_base;   // chunk-relative first item
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const unsigned char* W1 = reinterpret_cast<const unsigned char*>(a.w[0]);
  const unsigned char* W2 = reinterpret_cast<const unsigned char*>(a.w[1]);
  const unsigned char* W3 = reinterpret_cast<const unsigned char*>(a.w[2]);
  unsigned char* X3 = reinterpret_cast<unsigned char*>(a.x3);
  const float s8 = a.pix_s8;

  // frame staging: 441 16-byte chunks; thread t takes chunks t and t + 256
  const bool c2 = tid + kThreads < kFrameBytes / 16;
  auto fload = [&](const uint8_t* fr, uint4& u0, uint4& u1) {
    u0 = reinterpret_cast<const uint4*>(fr)[tid];
    if (c2) u1 = reinterpret_cast<const uint4*>(fr)[tid + kThreads];
  };
  auto fstore = [&](int buf, const uint4& u0, const uint4& u1) {
    Fr::stage16(&fs[buf][tid * 16 * EB], u0, s8);
    if (c2) Fr::stage16(&fs[buf][(tid + kThreads) * 16 * EB], u1, s8);
  };

  // conv1 weights (A operand): K step s covers stack channel s/2, kernel rows
  // 4(s&1)..+3; lane group g holds kernel row 4(s&1)+g (8 kw values)
  V w1[8][2];
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int j = 0; j < 2; ++j) w1[s][j] = Fr::ld(W1 + ((16 * j + r16) * 256 + 32 * s + 8 * g) * EB);
  float b1[2][4];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int q = 0; q < 4; ++q) b1[j][q] = a.bias[0][16 * j + 4 * g + q];

  // conv1 pixel operand of fragment f: output pixel 16f + r16, kernel row kh
  int poff[kF1];
#pragma unroll
  for (int i = 0; i < kF1; ++i) {
    const int f = wave + kWaves * i;
    const int p = (f < 25 ? f : 0) * 16 + r16;
    poff[i] = ((p / 20) * 4 * kFrame + (p % 20) * 4) * EB;
  }

  // ---- S: channels 0..2 of the group's shared stack ----
  const ItemDesc d0 = a.desc[i0];
  f32x4 S[kF1][2];
#pragma unroll
  for (int i = 0; i < kF1; ++i) S[i][0] = S[i][1] = f32x4{0.f, 0.f, 0.f, 0.f};
  {
    uint4 u0, u1;
    fload(d0.frame[0], u0, u1);
    fstore(0, u0, u1);
    fload(d0.frame[1], u0, u1);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < 2) {                       // stage channel c+1 while using channel c
        fstore((c + 1) & 1, u0, u1);
        if (c == 0) fload(d0.frame[2], u0, u1);
      }
#pragma unroll
      for (int i = 0; i < kF1; ++i) {
        if (wave + kWaves * i >= 25) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int s = 2 * c + h;
          const V pv = Fr::ld_pix(&fs[c & 1][poff[i] + (4 * h + g) * kFrame * EB]);
          S[i][0] = Fr::mma(w1[s][0], pv, S[i][0]);
          S[i][1] = Fr::mma(w1[s][1], pv, S[i][1]);
        }
      }
      __syncthreads();
    }
  }

  // per-item frames: item k's channel 3 goes to fs[k & 1]
  uint4 nu0, nu1;
  fload(a.desc[i0].frame[3], nu0, nu1);
  fstore(0, nu0, nu1);
  if (G > 1) fload(a.desc[i0 + 1].frame[3], nu0, nu1);
  __syncthreads();

  for (int r0 = 0; r0 < G; r0 += T) {
    const int nt = (G - r0) < T ? (G - r0) : T;

    // ---- conv1: S + channel 3 of each item -> x1 ----
    for (int t = 0; t < nt; ++t) {
      const int k = r0 + t;                               // item within the group
      if (k + 1 < G) fstore((k + 1) & 1, nu0, nu1);       // next item's frame, other buffer
      if (k + 2 < G) fload(a.desc[i0 + k + 2].frame[3], nu0, nu1);
      const unsigned char* fb = fs[k & 1];
#pragma unroll
      for (int i = 0; i < kF1; ++i) {
        const int f = wave + kWaves * i;
        if (f >= 25) continue;
        f32x4 c0 = S[i][0], c1 = S[i][1];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const V pv = Fr::ld_pix(&fb[poff[i] + (4 * h + g) * kFrame * EB]);
          c0 = Fr::mma(w1[6 + h][0], pv, c0);
          c1 = Fr::mma(w1[6 + h][1], pv, c1);
        }
        const int p = f * 16 + r16;
        const float sc = a.acc_scale[0], o8 = a.out_s8[0];
        Fr::st4(&x1[x1_off<P>(t, p, 4 * g)], fmaxf(c0[0] * sc + b1[0][0], 0.f), fmaxf(c0[1] * sc + b1[0][1], 0.f),
                fmaxf(c0[2] * sc + b1[0][2], 0.f), fmaxf(c0[3] * sc + b1[0][3], 0.f), o8);
        Fr::st4(&x1[x1_off<P>(t, p, 16 + 4 * g)], fmaxf(c1[0] * sc + b1[1][0], 0.f),
                fmaxf(c1[1] * sc + b1[1][1], 0.f), fmaxf(c1[2] * sc + b1[1][2], 0.f),
                fmaxf(c1[3] * sc + b1[1][3], 0.f), o8);
      }
      __syncthreads();     // x1 item t complete; fs[(k+1)&1] staged for the next item
    }

    // ---- conv2: x1 -> x2 (pixel rows = nt*81) ----
    {
      const int rows = nt * 81;
      f32x4 acc[F2W][4];
      int pb[F2W];
      bool ok[F2W];
#pragma unroll
      for (int i = 0; i < F2W; ++i) {
        const int r = (wave + kWaves * i) * 16 + r16;
        ok[i] = r < rows;
        const int rr = ok[i] ? r : 0;
        const int t = rr / 81, p = rr % 81;
        pb[i] = t * 400 + (p / 9) * 2 * 20 + (p % 9) * 2;     // item-major input pixel
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      V wc[4], wn[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) wc[j] = Fr::ld(W2 + ((16 * j + r16) * 512 + 8 * g) * EB);
#pragma unroll 2
      for (int s = 0; s < 16; ++s) {
        if (s + 1 < 16) {
#pragma unroll
          for (int j = 0; j < 4; ++j) wn[j] = Fr::ld(W2 + ((16 * j + r16) * 512 + 32 * (s + 1) + 8 * g) * EB);
        }
        const int U = 4 * s + g, kh = U >> 4, kw = (U >> 2) & 3, cg = U & 3;
#pragma unroll
        for (int i = 0; i < F2W; ++i) {
          if (wave + kWaves * i >= F2) continue;
          const int pp = pb[i] + kh * 20 + kw;             // t*400 + pixel
          const int t = pp / 400, p = pp - t * 400;
          const V pv = ok[i] ? Fr::ld(&x1[x1_off<P>(t, p, 8 * cg)]) : V{};
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = Fr::mma(wc[j], pv, acc[i][j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) wc[j] = wn[j];
      }
      const float sc = a.acc_scale[1], o8 = a.out_s8[1];
#pragma unroll
      for (int i = 0; i < F2W; ++i) {
        if (wave + kWaves * i >= F2 || !ok[i]) continue;
        const int r = (wave + kWaves * i) * 16 + r16;
        const int t = r / 81, p = r % 81;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = 16 * j + 4 * g;
          Fr::st4(&x2[x2_off<P>(t, p, n)], fmaxf(acc[i][j][0] * sc + a.bias[1][n], 0.f),
                  fmaxf(acc[i][j][1] * sc + a.bias[1][n + 1], 0.f), fmaxf(acc[i][j][2] * sc + a.bias[1][n + 2], 0.f),
                  fmaxf(acc[i][j][3] * sc + a.bias[1][n + 3], 0.f), o8);
        }
      }
    }
    __syncthreads();

    // ---- conv3: x2 -> x3 (HBM, channels-last [item][49][64]) ----
    {
      const int rows = nt * 49;
      f32x4 acc[F3W][4];
      int pb[F3W];
      bool ok[F3W];
#pragma unroll
      for (int i = 0; i < F3W; ++i) {
        const int r = (wave + kWaves * i) * 16 + r16;
        ok[i] = r < rows;
        const int rr = ok[i] ? r : 0;
        const int t = rr / 49, p = rr % 49;
        pb[i] = t * 81 + (p / 7) * 9 + (p % 7);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      V wc[4], wn[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) wc[j] = Fr::ld(W3 + ((16 * j + r16) * 576 + 8 * g) * EB);
#pragma unroll 2
      for (int s = 0; s < 18; ++s) {
        if (s + 1 < 18) {
#pragma unroll
          for (int j = 0; j < 4; ++j) wn[j] = Fr::ld(W3 + ((16 * j + r16) * 576 + 32 * (s + 1) + 8 * g) * EB);
        }
        const int U = 4 * s + g, kk = U >> 3, cg = U & 7;
#pragma unroll
        for (int i = 0; i < F3W; ++i) {
          if (wave + kWaves * i >= F3) continue;
          const int pp = pb[i] + (kk / 3) * 9 + kk % 3;     // t*81 + pixel
          const int t = pp / 81, p = pp - t * 81;
          const V pv = ok[i] ? Fr::ld(&x2[x2_off<P>(t, p, 8 * cg)]) : V{};
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = Fr::mma(wc[j], pv, acc[i][j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) wc[j] = wn[j];
      }
      const float sc = a.acc_scale[2], o8 = a.out_s8[2];
      const long long item_first = i0 + r0;
#pragma unroll
      for (int i = 0; i < F3W; ++i) {
        if (wave + kWaves * i >= F3 || !ok[i]) continue;
        const int r = (wave + kWaves * i) * 16 + r16;
        const long long row = (item_first + r / 49) * 49 + r % 49;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = 16 * j + 4 * g;
          Fr::st4(X3 + (row * 64 + n) * EB, fmaxf(acc[i][j][0] * sc + a.bias[2][n], 0.f),
                  fmaxf(acc[i][j][1] * sc + a.bias[2][n + 1], 0.f), fmaxf(acc[i][j][2] * sc + a.bias[2][n + 2], 0.f),
                  fmaxf(acc[i][j][3] * sc + a.bias[2][n + 3], 0.f), o8);
        }
      }
    }
    // No barrier needed here: the next round's conv1 writes x1 (last read by
    // conv2, before the barrier above) and fs (its own per-item barriers);
    // x2 is rewritten only after the next round's conv1 barriers, which every
    // wave reaches after its conv3 reads.
  }
}

}  // namespace

void launch_conv_fused(int prec, int T, const FusedConvArgs& a, int n_groups, hipStream_t s) {
  if (n_groups <= 0) return;
  dim3 grid((unsigned)n_groups), block(kThreads);
  if (prec == P_BF16) {   // BF16 at T = 4 exceeds the LDS of one CU: T <= 3
    if (T == 1) hipLaunchKernelGGL((conv_fused_kernel<P_BF16, 1>), grid, block, 0, s, a);
    else if (T == 2) hipLaunchKernelGGL((conv_fused_kernel<P_BF16, 2>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((conv_fused_kernel<P_BF16, 3>), grid, block, 0, s, a);
  } else {
    if (T == 1) hipLaunchKernelGGL((conv_fused_kernel<P_FP8, 1>), grid, block, 0, s, a);
    else if (T == 2) hipLaunchKernelGGL((conv_fused_kernel<P_FP8, 2>), grid, block, 0, s, a);
    else if (T == 4) hipLaunchKernelGGL((conv_fused_kernel<P_FP8, 4>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((conv_fused_kernel<P_FP8, 3>), grid, block, 0, s, a);
  }
}

}  // namespace bcts
