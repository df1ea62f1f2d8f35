// fc1 of the Nature-DQN on the matrix cores: H = ReLU(X W^T + b) with
// X [n][3136] (conv3 output, channels-last) and W [512][3136] (rows re-laid
// out to the same (h, w, c) order), BF16 or OCP e4m3 operands, FP32
// accumulate.  H [n][512] in the operand type feeds fc2.
//
// A workgroup of 8 wavefronts computes a 256 (stacks) x 256 (neurons) tile:
// wave (wm, wn) owns 64 x 128, i.e. 4 x 8 MFMA 16x16x32 fragments, so one
// LDS operand read feeds 4 or 8 MFMAs and each global byte feeds 256 output
// columns (the L2 -> CU path, not the matrix cores, bounds smaller tiles).  The K
// loop moves 64 K values per stage: the next stage's tiles are loaded from
// HBM/L2 into registers while the current stage's MFMAs run, then written to
// the other half of a double-buffered LDS, so one barrier separates stages.
// The product is computed transposed (D[neuron][stack] = W X^T) so each lane
// finishes with 4 consecutive neurons of one stack and stores them at once.
// Rows past n are clamped (read a valid row) and not stored.
#include "bcts_internal.h"

namespace bcts {
namespace {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

constexpr int kThreads = 512;
constexpr int kBM = 256, kBN = 256, kBK = 64, kK = 3136;
constexpr int kStages = kK / kBK;                 // 49
static_assert(512 / kBN == 2, "the workgroup mapping assumes 2 neuron tiles");

__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int P> struct FT;
template <> struct FT<P_BF16> {
  typedef bf16x8 V;
  static constexpr int EB = 2;
  __device__ static f32x4 mma(V a, V b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  __device__ static void st4(void* p, float a, float b, float c, float d, float) {
    const bf16x2 h0 = __builtin_convertvector(f32x2{a, b}, bf16x2);
    const bf16x2 h1 = __builtin_convertvector(f32x2{c, d}, bf16x2);
    *reinterpret_cast<uint2*>(p) = make_uint2(__builtin_bit_cast(unsigned, h0), __builtin_bit_cast(unsigned, h1));
  }
};
template <> struct FT<P_FP8> {
  typedef long V;
  static constexpr int EB = 1;
  __device__ static f32x4 mma(V a, V b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0); }
  __device__ static void st4(void* p, float a, float b, float c, float d, float s8) {
    a = fminf(fmaxf(a * s8, -448.f), 448.f);
    b = fminf(fmaxf(b * s8, -448.f), 448.f);
    c = fminf(fmaxf(c * s8, -448.f), 448.f);
    d = fminf(fmaxf(d * s8, -448.f), 448.f);
    const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    *reinterpret_cast<unsigned*>(p) = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, lo, true);
  }
};

template <int P>
__global__ void __launch_bounds__(kThreads, 1)
fc1_kernel(long long n, const unsigned char* __restrict__ X, const unsigned char* __restrict__ W,
           const float* __restrict__ bias, float acc_scale, float out_s8, unsigned char* __restrict__ H) {
  typedef FT<P> Ft;
  typedef typename Ft::V V;
  constexpr int EB = Ft::EB;
  constexpr int RB = kBK * EB;                    // bytes of one tile row per stage
  constexpr int RS = RB + 16;                     // LDS row stride: +16 B against bank conflicts
  constexpr int UB = 16;                          // bytes per 16-byte load unit
  constexpr int UPR = RB / UB;                    // units per row per stage
  constexpr int AU = kBM * UPR / kThreads;        // A units per thread per stage
  constexpr int BU = kBN * UPR / kThreads;        // B units per thread per stage
  constexpr int KS = kBK / 32;                    // MFMA K steps per stage
  __shared__ __attribute__((aligned(16))) unsigned char As[2][kBM * RS];
  __shared__ __attribute__((aligned(16))) unsigned char Bs[2][kBN * RS];

  // Workgroups are dealt to the 8 XCDs round-robin (XCD = id mod 8), each
  // with its own L2.  The 2 neuron tiles of one stack tile go to the same
  // XCD in consecutive slots, so its X tile is fetched from HBM once and
  // read by the other from that XCD's L2.  The grid is padded to a
  // multiple of 8 stack tiles; padding workgroups leave at once.
  const int bid = blockIdx.x, xcd = bid & 7, slot = bid >> 3;
  const long long mt = (long long)(slot >> 1) * 8 + xcd;
  if (mt * kBM >= n) return;
  const long long m0 = mt * kBM;
  const int n0 = (slot & 1) * kBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int wm = wave >> 1, wn = wave & 1;        // 4 x 2 waves

  // global -> register loads of stage st; unit u of a tile = (row u / UPR,
  // 16-byte column unit u % UPR)
#define FC1_GLOAD(st)                                                                                   \
  {                                                                                                     \
    _Pragma("unroll") for (int i = 0; i < AU; ++i) {                                                    \
      const int u = tid + i * kThreads, row = u / UPR, cu = u % UPR;                                    \
      long long m = m0 + row;                                                                           \
      if (m >= n) m = n - 1;                                                                            \
      ra[i] = *reinterpret_cast<const uint4*>(X + (m * kK + (long long)(st) * kBK) * EB + cu * UB);     \
    }                                                                                                   \
    _Pragma("unroll") for (int i = 0; i < BU; ++i) {                                                    \
      const int u = tid + i * kThreads, row = u / UPR, cu = u % UPR;                                    \
      rb[i] = *reinterpret_cast<const uint4*>(W + ((long long)(n0 + row) * kK + (long long)(st) * kBK) * EB + \
                                              cu * UB);                                                 \
    }                                                                                                   \
  }
#define FC1_LSTORE(buf)                                                                                 \
  {                                                                                                     \
    _Pragma("unroll") for (int i = 0; i < AU; ++i) {                                                    \
      const int u = tid + i * kThreads;                                                                 \
      *reinterpret_cast<uint4*>(&As[buf][(u / UPR) * RS + (u % UPR) * UB]) = ra[i];                     \
    }                                                                                                   \
    _Pragma("unroll") for (int i = 0; i < BU; ++i) {                                                    \
      const int u = tid + i * kThreads;                                                                 \
      *reinterpret_cast<uint4*>(&Bs[buf][(u / UPR) * RS + (u % UPR) * UB]) = rb[i];                     \
    }                                                                                                   \
  }
  uint4 ra[AU], rb[BU];

  f32x4 acc[8][4];            // [neuron frag][stack frag]
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  FC1_GLOAD(0);
  FC1_LSTORE(0);
  lds_barrier();
  for (int st = 0; st < kStages; ++st) {
    const int buf = st & 1;
    if (st + 1 < kStages) FC1_GLOAD(st + 1);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      V xv[4];
      const int kb = (ks * 32 + 8 * g) * EB;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        xv[j] = *reinterpret_cast<const V*>(&As[buf][(wm * 64 + j * 16 + r16) * RS + kb]);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const V wv = *reinterpret_cast<const V*>(&Bs[buf][(wn * 128 + i * 16 + r16) * RS + kb]);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Ft::mma(wv, xv[j], acc[i][j]);
      }
    }
    if (st + 1 < kStages) FC1_LSTORE(buf ^ 1);
    lds_barrier();
  }
#undef FC1_GLOAD
#undef FC1_LSTORE

  // epilogue: lane holds neurons n0 + wn*128 + 16i + 4g + q of stack m0 + wm*64 + 16j + r16
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int nb = n0 + wn * 128 + 16 * i + 4 * g;
    const float b0 = bias[nb], b1 = bias[nb + 1], b2 = bias[nb + 2], b3 = bias[nb + 3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long m = m0 + wm * 64 + 16 * j + r16;
      if (m < n)
        Ft::st4(H + (m * 512 + nb) * EB, fmaxf(acc[i][j][0] * acc_scale + b0, 0.f),
                fmaxf(acc[i][j][1] * acc_scale + b1, 0.f), fmaxf(acc[i][j][2] * acc_scale + b2, 0.f),
                fmaxf(acc[i][j][3] * acc_scale + b3, 0.f), out_s8);
    }
  }
}

}  // namespace

void launch_fc1_mfma(int prec, long long n, const void* x3, const void* w, const float* bias, float acc_scale,
                     float out_s8, void* h, hipStream_t s) {
  if (n <= 0) return;
  const long long mtiles = ((n + kBM - 1) / kBM + 7) / 8 * 8;
  dim3 grid((unsigned)(mtiles * (512 / kBN))), block(kThreads);
  const unsigned char* X = reinterpret_cast<const unsigned char*>(x3);
  const unsigned char* Wp = reinterpret_cast<const unsigned char*>(w);
  unsigned char* H = reinterpret_cast<unsigned char*>(h);
  if (prec == P_BF16) hipLaunchKernelGGL((fc1_kernel<P_BF16>), grid, block, 0, s, n, X, Wp, bias, acc_scale, out_s8, H);
  else hipLaunchKernelGGL((fc1_kernel<P_FP8>), grid, block, 0, s, n, X, Wp, bias, acc_scale, out_s8, H);
}

}  // namespace bcts
