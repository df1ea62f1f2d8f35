// Nature-DQN value network over a chunk of eval items, as implicit GEMMs on
// the CDNA4 matrix cores (the leaf-scoring step of Alg. 1).
//
// Every layer is C[M][N] = act(scale * A[M][K] B[K][N] + bias) with the
// activations kept channels-last (NHWC), so that the GEMM output of one layer
// is, row-major, the next layer's input tensor:
//
//   layer  rows per item      N    K = unit order (8 K values per unit)
//   conv1  20*20 (oy, ox)     32   256 = (c, kh) x kw[8]     from 4 uint8 frames
//   conv2   9*9               64   512 = (kh, kw, c/8) x 8   from x1 [20][20][32]
//   conv3   7*7               64   576 = (kh, kw, c/8) x 8   from x2 [9][9][64]
//   fc1     1                512  3136 = (h, w, c/8) x 8     from x3 [7][7][64]
//   fc2     1                 32   512                       from h [512]; max over A
//
// A workgroup (4 wavefronts) computes a BM x BN tile: im2col rows are
// gathered unit by unit (8 contiguous K values per load) into LDS, weights
// W[N][K] likewise, then each wavefront runs 16x16 MFMAs over its 32-row
// slice.  Operands: FP32 (v_mfma_f32_16x16x4_f32), BF16
// (v_mfma_f32_16x16x32_bf16) or OCP e4m3 (v_mfma_f32_16x16x32_fp8_fp8), all
// accumulating in FP32.  The 1/255 input scaling is applied to conv1's
// accumulator; FP8 layers rescale by 1/(input scale * weight scale).
#include <type_traits>

#include "bcts_internal.h"
#include "qnet_groups.h"

namespace bcts {
namespace {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

constexpr int kThreads = 256;
constexpr int kBM = 128;       // rows per workgroup tile
constexpr int kBKU = 4;        // K units (of 8) per LDS stage: 32 K values

// Barrier for LDS hand-offs only: unlike __syncthreads() it does not wait for
// outstanding global loads, so the next stage's prefetch stays in flight.
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// ---- element types ------------------------------------------------------
template <int P> struct PT;
template <> struct PT<P_FP32> { typedef float T; };
template <> struct PT<P_BF16> { typedef uint16_t T; };
template <> struct PT<P_FP8> { typedef uint8_t T; };

__device__ __forceinline__ uint16_t f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);             // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

// float -> OCP e4m3 (saturating to +-448), round to nearest even
__device__ __forceinline__ uint8_t f2e4m3(float f) {
  f = fminf(fmaxf(f, -448.f), 448.f);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(f, 0.f, 0, false);
  return (uint8_t)(w & 0xFF);
}

// A unit: 8 consecutive K values of one GEMM row, in the operand type.
template <int P> struct Unit;
template <> struct Unit<P_FP32> { float4 a, b; };
template <> struct Unit<P_BF16> { uint4 v; };
template <> struct Unit<P_FP8> { uint2 v; };

template <int P> __device__ __forceinline__ Unit<P> zero_unit();
template <> __device__ __forceinline__ Unit<P_FP32> zero_unit<P_FP32>() {
  Unit<P_FP32> u; u.a = make_float4(0, 0, 0, 0); u.b = u.a; return u;
}
template <> __device__ __forceinline__ Unit<P_BF16> zero_unit<P_BF16>() {
  Unit<P_BF16> u; u.v = make_uint4(0, 0, 0, 0); return u;
}
template <> __device__ __forceinline__ Unit<P_FP8> zero_unit<P_FP8>() {
  Unit<P_FP8> u; u.v = make_uint2(0, 0); return u;
}

// load 8 elements of the layer's own type
template <int P> __device__ __forceinline__ Unit<P> load_unit(const typename PT<P>::T* p);
template <> __device__ __forceinline__ Unit<P_FP32> load_unit<P_FP32>(const float* p) {
  Unit<P_FP32> u;
  u.a = *reinterpret_cast<const float4*>(p);
  u.b = *reinterpret_cast<const float4*>(p + 4);
  return u;
}
template <> __device__ __forceinline__ Unit<P_BF16> load_unit<P_BF16>(const uint16_t* p) {
  Unit<P_BF16> u; u.v = *reinterpret_cast<const uint4*>(p); return u;
}
template <> __device__ __forceinline__ Unit<P_FP8> load_unit<P_FP8>(const uint8_t* p) {
  Unit<P_FP8> u; u.v = *reinterpret_cast<const uint2*>(p); return u;
}

// 8 pixels (two little-endian words of uint8) -> operand unit; fp8 scales the pixel
template <int P> __device__ __forceinline__ Unit<P> pix_cvt(unsigned w0, unsigned w1, float s8);
template <> __device__ __forceinline__ Unit<P_FP32> pix_cvt<P_FP32>(unsigned w0, unsigned w1, float) {
  Unit<P_FP32> u;
  u.a = make_float4((float)(w0 & 255u), (float)((w0 >> 8) & 255u), (float)((w0 >> 16) & 255u),
                    (float)(w0 >> 24));
  u.b = make_float4((float)(w1 & 255u), (float)((w1 >> 8) & 255u), (float)((w1 >> 16) & 255u),
                    (float)(w1 >> 24));
  return u;
}
__device__ __forceinline__ unsigned pack_bf2(unsigned a, unsigned b) {
  // integers 0..255 are exact in bf16: the float's top 16 bits
  return (__float_as_uint((float)a) >> 16) | (__float_as_uint((float)b) & 0xFFFF0000u);
}
template <> __device__ __forceinline__ Unit<P_BF16> pix_cvt<P_BF16>(unsigned w0, unsigned w1, float) {
  Unit<P_BF16> u;
  u.v.x = pack_bf2(w0 & 255u, (w0 >> 8) & 255u);
  u.v.y = pack_bf2((w0 >> 16) & 255u, w0 >> 24);
  u.v.z = pack_bf2(w1 & 255u, (w1 >> 8) & 255u);
  u.v.w = pack_bf2((w1 >> 16) & 255u, w1 >> 24);
  return u;
}
template <> __device__ __forceinline__ Unit<P_FP8> pix_cvt<P_FP8>(unsigned w0, unsigned w1, float s8) {
  unsigned o[2];
  const unsigned w[2] = {w0, w1};
  for (int h = 0; h < 2; ++h) {
    int lo = __builtin_amdgcn_cvt_pk_fp8_f32(fminf((float)(w[h] & 255u) * s8, 448.f),
                                             fminf((float)((w[h] >> 8) & 255u) * s8, 448.f), 0, false);
    int hi = __builtin_amdgcn_cvt_pk_fp8_f32(fminf((float)((w[h] >> 16) & 255u) * s8, 448.f),
                                             fminf((float)(w[h] >> 24) * s8, 448.f), lo, true);
    o[h] = (unsigned)hi;
  }
  Unit<P_FP8> u; u.v = make_uint2(o[0], o[1]); return u;
}
// 8 pixels at p (4-byte aligned)
template <int P> __device__ __forceinline__ Unit<P> pix_unit(const uint8_t* p, float s8) {
  return pix_cvt<P>(*reinterpret_cast<const unsigned*>(p), *reinterpret_cast<const unsigned*>(p + 4), s8);
}

// ---- layer geometry -----------------------------------------------------
template <int L> struct Geo;
template <> struct Geo<0> { static constexpr int MPI = 400, N = 32, K = 256, BN = 32; };
template <> struct Geo<1> { static constexpr int MPI = 81, N = 64, K = 512, BN = 64; };
template <> struct Geo<2> { static constexpr int MPI = 49, N = 64, K = 576, BN = 64; };
template <> struct Geo<3> { static constexpr int MPI = 1, N = 512, K = 3136, BN = 128; };
template <> struct Geo<4> { static constexpr int MPI = 1, N = 32, K = 512, BN = 32; };

// Per-thread view of one GEMM row: where its units come from.
struct RowSrc {
  const void* base;            // layer input of the row's item (frame 0 for conv1)
  const uint8_t* fr[4];        // conv1: the 4 frames
  int off;                     // element offset of the row's window origin
  bool valid;
};

template <int L, int P>
__device__ __forceinline__ RowSrc row_src(long long m, long long M, const ItemDesc* desc,
                                          const typename PT<P>::T* in) {
  RowSrc r;
  r.valid = m < M;
  if (!r.valid) m = 0;
  const long long item = m / Geo<L>::MPI;
  const int pix = (int)(m - item * Geo<L>::MPI);
  if (L == 0) {
    const ItemDesc& d = desc[item];
    for (int c = 0; c < 4; ++c) r.fr[c] = d.frame[c];
    const int oy = pix / 20, ox = pix % 20;
    r.off = oy * 4 * kFrame + ox * 4;
    r.base = nullptr;
  } else if (L == 1) {
    const int oy = pix / 9, ox = pix % 9;
    r.base = in + item * 12800;
    r.off = (oy * 2 * 20 + ox * 2) * 32;
  } else if (L == 2) {
    const int oy = pix / 7, ox = pix % 7;
    r.base = in + item * 5184;
    r.off = (oy * 9 + ox) * 64;
  } else if (L == 3) {
    r.base = in + item * 3136;
    r.off = 0;
  } else {
    r.base = in + item * 512;
    r.off = 0;
  }
  return r;
}

template <int L, int P>
__device__ __forceinline__ Unit<P> gather(const RowSrc& r, int U, float s8) {
  typedef typename PT<P>::T T;
  if (!r.valid) return zero_unit<P>();
  if (L == 0) {
    const int c = U >> 3, kh = U & 7;
    return pix_unit<P>(r.fr[c] + r.off + kh * kFrame, s8);
  } else if (L == 1) {
    const int kh = U >> 4, kw = (U >> 2) & 3, cg = U & 3;
    return load_unit<P>((const T*)r.base + r.off + (kh * 20 + kw) * 32 + cg * 8);
  } else if (L == 2) {
    const int kk = U >> 3, cg = U & 7, kh = kk / 3, kw = kk % 3;
    return load_unit<P>((const T*)r.base + r.off + (kh * 9 + kw) * 64 + cg * 8);
  } else {
    return load_unit<P>((const T*)r.base + U * 8);
  }
}

// ---- LDS tiles ----------------------------------------------------------
// Row stride in elements: 32 K values plus padding against bank conflicts.
template <int P> struct Lds;
template <> struct Lds<P_FP32> { static constexpr int S = 33; };
template <> struct Lds<P_BF16> { static constexpr int S = 40; };
template <> struct Lds<P_FP8> { static constexpr int S = 48; };

template <int P>
__device__ __forceinline__ void st_unit(typename PT<P>::T* row, int u, const Unit<P>& v);
template <> __device__ __forceinline__ void st_unit<P_FP32>(float* row, int u, const Unit<P_FP32>& v) {
  float* d = row + u * 8;     // stride 33 breaks 16-byte alignment: scalar stores
  d[0] = v.a.x; d[1] = v.a.y; d[2] = v.a.z; d[3] = v.a.w;
  d[4] = v.b.x; d[5] = v.b.y; d[6] = v.b.z; d[7] = v.b.w;
}
template <> __device__ __forceinline__ void st_unit<P_BF16>(uint16_t* row, int u, const Unit<P_BF16>& v) {
  *reinterpret_cast<uint4*>(row + u * 8) = v.v;
}
template <> __device__ __forceinline__ void st_unit<P_FP8>(uint8_t* row, int u, const Unit<P_FP8>& v) {
  *reinterpret_cast<uint2*>(row + u * 8) = v.v;
}

// One 32-K stage of MFMAs for a wavefront's 32 x BN slice.
template <int P, int NF>
__device__ __forceinline__ void mma_stage(const typename PT<P>::T* As, const typename PT<P>::T* Bs,
                                          int lane, f32x4 (&acc)[2][NF]) {
  constexpr int S = Lds<P>::S;
  const int r = lane & 15, g = lane >> 4;
  if constexpr (P == P_FP32) {
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      float a[2], b[NF];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[(i * 16 + r) * S + ks * 4 + g];
#pragma unroll
      for (int j = 0; j < NF; ++j) b[j] = Bs[(j * 16 + r) * S + ks * 4 + g];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  } else if constexpr (P == P_BF16) {
    bf16x8 a[2], b[NF];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(As + (i * 16 + r) * S + g * 8);
#pragma unroll
    for (int j = 0; j < NF; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(Bs + (j * 16 + r) * S + g * 8);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  } else {
    long a[2], b[NF];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const long*>(As + (i * 16 + r) * S + g * 8);
#pragma unroll
    for (int j = 0; j < NF; ++j)
      b[j] = *reinterpret_cast<const long*>(Bs + (j * 16 + r) * S + g * 8);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

template <int P> __device__ __forceinline__ void st_out(typename PT<P>::T* p, float v, float s8);
template <> __device__ __forceinline__ void st_out<P_FP32>(float* p, float v, float) { *p = v; }
template <> __device__ __forceinline__ void st_out<P_BF16>(uint16_t* p, float v, float) { *p = f2bf(v); }
template <> __device__ __forceinline__ void st_out<P_FP8>(uint8_t* p, float v, float s8) { *p = f2e4m3(v * s8); }

struct LayerArgs {
  long long M;                 // rows = items * rows per item
  const ItemDesc* desc;
  const void* in;              // layer input (conv2..fc2)
  const void* w;               // W[N][K] in operand type
  const float* bias;
  float acc_scale;             // multiplies the accumulator before the bias
  float in_s8;                 // fp8: scale applied to the layer input (conv1 pixels)
  float out_s8;                // fp8: scale of the next layer's input
  void* out;                   // C (conv1..fc1)
  float* V;                    // fc2: max_a Q per item
  float* q0;                   // fc2: [n_roots][18]
  float* part;                 // FP32 fc1: the K slices' partial sums [kFc1Split][M][512]
  const FusedGroup* groups;    // conv1 by sibling groups: the chunk's groups
  int n_groups;
  long long item_base;         // plan-global index of the chunk's first item
};

template <int L, int P, bool WK = false>
__global__ void __launch_bounds__(kThreads) layer_kernel(LayerArgs args) {
  typedef typename PT<P>::T T;
  constexpr int BN = Geo<L>::BN, NF = BN / 16, K = Geo<L>::K, NU = K / 8;
  constexpr int S = Lds<P>::S;
  constexpr int NSTAGE = NU / kBKU;
  static_assert(NU % kBKU == 0, "K must be a multiple of 32");
  __shared__ __attribute__((aligned(16))) T As[kBM * S];
  __shared__ __attribute__((aligned(16))) T Bs[BN * S];
  __shared__ float Cs[(L == 4) ? kBM * 33 : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long m0 = (long long)blockIdx.x * kBM;
  const int n0 = blockIdx.y * BN;
  const T* W = reinterpret_cast<const T*>(args.w);
  const T* in = reinterpret_cast<const T*>(args.in);

  // A: thread owns rows ra, ra + 64 and unit ua of each stage
  const int ra = tid >> 2, ua = tid & 3;
  RowSrc rs0 = row_src<L, P>(m0 + ra, args.M, args.desc, in);
  RowSrc rs1 = row_src<L, P>(m0 + ra + 64, args.M, args.desc, in);
  // B: BN rows x 4 units; thread t < BN*4 owns row t>>2 (and +64 for BN=128)
  constexpr int BPASS = (BN * kBKU + kThreads - 1) / kThreads;

  f32x4 acc[2][NF];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  Unit<P> ga0, ga1, gb[BPASS];
  auto gload = [&](int st) {
    const int U = st * kBKU + ua;
    ga0 = gather<L, P>(rs0, U, args.in_s8);
    ga1 = gather<L, P>(rs1, U, args.in_s8);
#pragma unroll
    for (int p = 0; p < BPASS; ++p) {
      const int t = tid + p * kThreads;
      if (t < BN * kBKU) {
        const int n = t >> 2, u = t & 3;
        gb[p] = load_unit<P>(W + (long long)(n0 + n) * K + (st * kBKU + u) * 8);
      }
    }
  };
  auto lstore = [&]() {
    st_unit<P>(As + ra * S, ua, ga0);
    st_unit<P>(As + (ra + 64) * S, ua, ga1);
#pragma unroll
    for (int p = 0; p < BPASS; ++p) {
      const int t = tid + p * kThreads;
      if (t < BN * kBKU) st_unit<P>(Bs + (t >> 2) * S, t & 3, gb[p]);
    }
  };

  // FP32 fc1 runs K in kFc1Split slices, each summed from zero; the slices'
  // sums are added in slice order.  Either one workgroup per slice
  // (blockIdx.z) and fc1_reduce_kernel adds them, or (WK, for chunks with
  // workgroups enough without the split) each workgroup runs
  // the slices in turn and adds them in registers: the same sums in the
  // same order, the same bits (see run_layer).
  constexpr bool kSplit = (L == 3 && P == P_FP32);
  static_assert(!kSplit || NSTAGE % kFc1Split == 0, "fc1's stages split evenly");
  constexpr bool whole_k = kSplit && WK;
  const int nz = whole_k ? kFc1Split : 1;
  f32x4 tot[2][NF];
  for (int zi = 0; zi < nz; ++zi) {
    const int z = whole_k ? zi : (int)blockIdx.z;
    const int st0 = kSplit ? z * (NSTAGE / kFc1Split) : 0;
    const int st1 = kSplit ? st0 + NSTAGE / kFc1Split : NSTAGE;
    if (zi > 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    gload(st0);
    lstore();
    lds_barrier();
    for (int st = st0; st < st1; ++st) {
      if (st + 1 < st1) gload(st + 1);
      mma_stage<P, NF>(As + wave * 32 * S, Bs, lane, acc);
      lds_barrier();
      if (st + 1 < st1) {
        lstore();
        lds_barrier();
      }
    }
    if constexpr (whole_k) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j) tot[i][j] = zi == 0 ? acc[i][j] : tot[i][j] + acc[i][j];
    }
  }

  // epilogue: lane holds rows 4*(lane>>4) + q, column lane & 15 of each frag
  const int col = lane & 15, rq = (lane >> 4) * 4;
  if constexpr (whole_k) {
    // h = ReLU(sum * scale + b), as fc1_reduce_kernel forms it
    float* out = reinterpret_cast<float*>(args.out);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        const int n = n0 + j * 16 + col;
        const float b = args.bias[n];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const long long m = m0 + wave * 32 + i * 16 + rq + q;
          if (m < args.M) out[m * Geo<L>::N + n] = fmaxf(fmaf(tot[i][j][q], args.acc_scale, b), 0.f);
        }
      }
  } else if constexpr (kSplit) {
    // the slice's raw partial sums; fc1_reduce_kernel adds the slices in order
    float* part = args.part + (long long)blockIdx.z * args.M * Geo<L>::N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        const int n = n0 + j * 16 + col;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const long long m = m0 + wave * 32 + i * 16 + rq + q;
          if (m < args.M) part[m * Geo<L>::N + n] = acc[i][j][q];
        }
      }
  } else if constexpr (L < 4) {
    T* out = reinterpret_cast<T*>(args.out);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        const int n = n0 + j * 16 + col;
        const float b = args.bias[n];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const long long m = m0 + wave * 32 + i * 16 + rq + q;
          if (m < args.M) {
            float v = fmaxf(acc[i][j][q] * args.acc_scale + b, 0.f);
            st_out<P>(out + m * Geo<L>::N + n, v, args.out_s8);
          }
        }
      }
  } else {
    // fc2: Q = acc * scale + b; V = max over the item's A actions
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        const int n = j * 16 + col;
        const float b = n < kMaxA ? args.bias[n] : 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          Cs[(wave * 32 + i * 16 + rq + q) * 33 + n] = acc[i][j][q] * args.acc_scale + b;
      }
    lds_barrier();
    if (tid < kBM) {
      const long long m = m0 + tid;
      if (m < args.M) {
        const ItemDesc& d = args.desc[m];
        const float* row = Cs + tid * 33;
        float v = row[0];
        for (int a = 1; a < d.A; ++a) v = fmaxf(v, row[a]);
        args.V[m] = v;
        if (d.q0_root >= 0)
          for (int a = 0; a < kMaxA; ++a) args.q0[(long long)d.q0_root * kMaxA + a] = row[a];
      }
    }
  }
}

// One 32-K stage of MFMAs for a wavefront's 32 x (16 NF) slice of conv1
// with the A operand as raw pixel bytes (row stride kS8 bytes), converted
// to the operand type as it is read: the same operand values as mma_stage
// on a converted tile, in a quarter of the LDS (FP32).
constexpr int kS8 = 40;        // bytes per pixel row of a stage: 32 + 8 against bank conflicts
template <int P, int NF>
__device__ __forceinline__ void mma_stage_pix(const uint8_t* A8, const typename PT<P>::T* Bs, int lane, float s8,
                                              f32x4 (&acc)[2][NF]) {
  constexpr int S = Lds<P>::S;
  const int r = lane & 15, g = lane >> 4;
  if constexpr (P == P_FP32) {
    // FP32 rows are stored by lane group: bytes 8g .. 8g + 7 hold K values
    // 4 ks + g, ks = 0..7, the values lane group g feeds the 8 MFMA steps
    uint2 w[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) w[i] = *reinterpret_cast<const uint2*>(A8 + (i * 16 + r) * kS8 + g * 8);
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      float a[2], b[NF];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = (float)(((ks < 4 ? w[i].x : w[i].y) >> (8 * (ks & 3))) & 255u);
#pragma unroll
      for (int j = 0; j < NF; ++j) b[j] = Bs[(j * 16 + r) * S + ks * 4 + g];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  } else {
    typename std::conditional<P == P_BF16, bf16x8, long>::type a[2], b[NF];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint2 w = *reinterpret_cast<const uint2*>(A8 + (i * 16 + r) * kS8 + g * 8);
      const Unit<P> u = pix_cvt<P>(w.x, w.y, s8);
      __builtin_memcpy(&a[i], &u, sizeof(a[i]));
    }
#pragma unroll
    for (int j = 0; j < NF; ++j) __builtin_memcpy(&b[j], Bs + (j * 16 + r) * S + g * 8, sizeof(b[j]));
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        if constexpr (P == P_BF16)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        else
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[i], b[j], acc[i][j], 0, 0, 0);
      }
  }
}

// conv1 over sibling groups.  The stacks of a group (the A children of one
// node in Alg. 1's leaf level, the A depth-1 nodes of a root) hold the same
// channels 0..2, so conv1's sum over them, K units 0..23 (stages 0..5), is
// the same for every sibling.  A workgroup takes 128 rows of (group, output
// pixel) -- at most two groups, since a group has 400 -- sums the shared
// stages once, then for each sibling adds channel 3 (stages 6 and 7) to a
// copy of that partial sum and stores the sibling's rows.  Every output sees
// the MFMAs of layer_kernel<0, P> in the same order, so the two agree bit
// for bit; the work per group of A falls from 8A stages to 6 + 2A.  The
// pixel tiles hold raw bytes (converted as the MFMAs read them) and are
// double-buffered: one barrier per stage.
template <int P>
__global__ void __launch_bounds__(kThreads) conv1_groups_kernel(LayerArgs args) {
  typedef typename PT<P>::T T;
  constexpr int S = Lds<P>::S, N = Geo<0>::N, NF = N / 16, K = Geo<0>::K, PIX = Geo<0>::MPI;
  constexpr int kShared = 6;                    // stages over channels 0..2
  static_assert(Geo<0>::BN == N && K == 8 * kBKU * 8, "conv1: one column tile, 8 stages");
  __shared__ __attribute__((aligned(16))) uint8_t A8[2][kBM * kS8];   // pixel bytes, double-buffered
  __shared__ __attribute__((aligned(16))) T Bs[2][N * S];      // the shared stages' weights, double-buffered
  __shared__ __attribute__((aligned(16))) T Bo[2][N * S];      // channel 3's two stages, resident
  __shared__ const uint8_t* own[2][kMaxA];                     // each sibling's channel-3 frame
  __shared__ const uint8_t* shf[2][3];                         // the two groups' channels 0..2

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int M = (int)args.M;                    // n_groups * 400 rows (< 2^31: checked by the launcher)
  const int m0 = (int)blockIdx.x * kBM;
  const int g_lo = m0 / PIX;
  const int split = (g_lo + 1) * PIX - m0;      // the tile's rows in group g_lo
  const bool has_hi = split < kBM && g_lo + 1 < args.n_groups;
  const FusedGroup glo = args.groups[g_lo];
  const int i_lo = (int)(glo.item0 - args.item_base), c_lo = glo.count;
  int i_hi = i_lo, c_hi = 0;
  if (has_hi) {
    const FusedGroup ghi = args.groups[g_lo + 1];
    i_hi = (int)(ghi.item0 - args.item_base);
    c_hi = ghi.count;
  }
  const int smax = c_lo > c_hi ? c_lo : c_hi;
  const T* W = reinterpret_cast<const T*>(args.w);

  if (tid < 2 * kMaxA) {
    const int h = tid / kMaxA, sb = tid - h * kMaxA;
    own[h][sb] = sb < (h ? c_hi : c_lo) ? args.desc[(h ? i_hi : i_lo) + sb].frame[3] : nullptr;
  } else if (tid < 2 * kMaxA + 6) {
    const int h = (tid - 2 * kMaxA) / 3, c = (tid - 2 * kMaxA) % 3;
    shf[h][c] = args.desc[h ? i_hi : i_lo].frame[c];
  }
  {
    // channel 3's weights: units 24..31 of every column, one per thread
    const int n = tid >> 3, u = tid & 7;
    st_unit<P>(Bo[u >> 2] + n * S, u & 3, load_unit<P>(W + (long long)n * K + (3 * 8 + u) * 8));
  }
  lds_barrier();

  // A: thread owns rows ra, ra + 64 and unit ua of each stage; a row is
  // (group g_lo + h, output pixel), its window origin at `off` (-1: past M)
  const int ra = tid >> 2, ua = tid & 3;
  int off[2], hr[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int r = ra + 64 * k, m = m0 + r;
    hr[k] = r >= split;
    const int pix = m - (g_lo + hr[k]) * PIX;
    off[k] = m < M ? (pix / 20) * 4 * kFrame + (pix % 20) * 4 : -1;
  }
  uint2 raw[2];
  Unit<P> gb;
  // shared stage t: channel t / 2 of the row's group, rows kh = 4 (t % 2) + ua
  auto load_shared = [&](int t) {
    const int U = t * kBKU + ua, c = U >> 3, kh = U & 7;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      raw[k] = make_uint2(0u, 0u);
      if (off[k] >= 0) {
        const uint8_t* q = shf[hr[k]][c] + off[k] + kh * kFrame;
        raw[k] = make_uint2(*reinterpret_cast<const unsigned*>(q), *reinterpret_cast<const unsigned*>(q + 4));
      }
    }
    if (tid < N * kBKU) gb = load_unit<P>(W + (long long)(tid >> 2) * K + (t * kBKU + (tid & 3)) * 8);
  };
  // channel-3 stage hf (0, 1) of sibling sb
  auto load_own = [&](int sb, int hf) {
    const int kh = hf * kBKU + ua;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      raw[k] = make_uint2(0u, 0u);
      const uint8_t* f = own[hr[k]][sb];
      if (off[k] >= 0 && f) {                   // else past M or past the row's group
        const uint8_t* q = f + off[k] + kh * kFrame;
        raw[k] = make_uint2(*reinterpret_cast<const unsigned*>(q), *reinterpret_cast<const unsigned*>(q + 4));
      }
    }
  };
  auto store_a = [&](int buf) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      uint8_t* row = &A8[buf][(ra + 64 * k) * kS8];
      if constexpr (P == P_FP32) {
        // K value 8 ua + e goes to lane group e % 4, step 2 ua + e / 4
        const unsigned lo = __builtin_amdgcn_perm(raw[k].y, raw[k].x, 0x05010400u);   // x0 y0 x1 y1
        const unsigned hi = __builtin_amdgcn_perm(raw[k].y, raw[k].x, 0x07030602u);   // x2 y2 x3 y3
        *reinterpret_cast<uint16_t*>(row + 0 * 8 + 2 * ua) = (uint16_t)lo;
        *reinterpret_cast<uint16_t*>(row + 1 * 8 + 2 * ua) = (uint16_t)(lo >> 16);
        *reinterpret_cast<uint16_t*>(row + 2 * 8 + 2 * ua) = (uint16_t)hi;
        *reinterpret_cast<uint16_t*>(row + 3 * 8 + 2 * ua) = (uint16_t)(hi >> 16);
      } else {
        *reinterpret_cast<uint2*>(row + ua * 8) = raw[k];
      }
    }
  };
  auto store_b = [&](int buf) {
    if (tid < N * kBKU) st_unit<P>(Bs[buf] + (tid >> 2) * S, tid & 3, gb);
  };
  const uint8_t* Aw[2] = {A8[0] + wave * 32 * kS8, A8[1] + wave * 32 * kS8};

  f32x4 acc[2][NF], part[2][NF];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // shared stages: stage t in buffer t % 2; a buffer is refilled only after
  // the barrier that follows every wavefront's reads of it
  load_shared(0);
  store_a(0);
  store_b(0);
  lds_barrier();
  for (int t = 0; t < kShared; ++t) {
    if (t + 1 < kShared) load_shared(t + 1);
    else load_own(0, 0);
    mma_stage_pix<P, NF>(Aw[t & 1], Bs[t & 1], lane, args.in_s8, acc);
    store_a((t + 1) & 1);
    if (t + 1 < kShared) store_b((t + 1) & 1);
    lds_barrier();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) part[i][j] = acc[i][j];

  // siblings: channel 3 (stages 6 and 7, buffers 0 and 1) on a copy of the
  // partial sum, then the sibling's rows.
  // Row index of the output: item * 400 + pix = m + (i_h - g_h) * 400.
  const int col = lane & 15, rq = (lane >> 4) * 4;
  const int d_lo = (i_lo - g_lo) * PIX, d_hi = (i_hi - g_lo - 1) * PIX;
  T* out = reinterpret_cast<T*>(args.out);
  for (int sb = 0; sb < smax; ++sb) {
    load_own(sb, 1);
    mma_stage_pix<P, NF>(Aw[0], Bo[0], lane, args.in_s8, acc);
    store_a(1);
    lds_barrier();
    const bool more = sb + 1 < smax;
    if (more) load_own(sb + 1, 0);
    mma_stage_pix<P, NF>(Aw[1], Bo[1], lane, args.in_s8, acc);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = wave * 32 + i * 16 + rq + q, m = m0 + rr;
        const int h = rr >= split;
        if (m < M && sb < (h ? c_hi : c_lo)) {
          T* o = out + (long long)(m + (h ? d_hi : d_lo) + sb * PIX) * N + col;
#pragma unroll
          for (int j = 0; j < NF; ++j) {
            const float v = fmaxf(acc[i][j][q] * args.acc_scale + args.bias[j * 16 + col], 0.f);
            st_out<P>(o + j * 16, v, args.out_s8);
          }
        }
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) acc[i][j] = part[i][j];
    if (more) store_a(0);
    lds_barrier();
  }
}

// FP32 fc1: h = ReLU((part_0 + part_1 + ... in slice order) * scale + b)
__global__ void fc1_reduce_kernel(long long M, const float* __restrict__ part, const float* __restrict__ bias,
                                  float scale, float* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * 512) return;
  float v = part[t];
  for (int z = 1; z < kFc1Split; ++z) v += part[z * M * 512 + t];
  out[t] = fmaxf(fmaf(v, scale, bias[t % 512]), 0.f);
}

// FP32 fc1 (K = 3136, 98 stages) splits K into kFc1Split slices summed in a
// fixed order, so that every row's sum order stays fixed whatever the
// batch.  A small batch (the correction's FP32 evaluations of a few roots)
// runs each slice as its own workgroup, 7x more workgroups than one long
// serial K loop, and a second kernel adds the slices; a chunk that fills
// the GPU without that runs all slices in each workgroup and adds them in
// registers, sparing the partial sums' round trip through HBM.
template <int L, int P>
void run_layer(const LayerArgs& a, hipStream_t s) {
  const long long blocks = (a.M + kBM - 1) / kBM;
  constexpr bool split_k = (L == 3 && P == P_FP32);
  // slices as workgroups only while the chunk's own workgroups (4 per 128
  // stacks) fall short of about two per CU
  const bool split = split_k && blocks * (Geo<L>::N / Geo<L>::BN) < 512;
  dim3 grid((unsigned)blocks, Geo<L>::N / Geo<L>::BN, split ? kFc1Split : 1);
  if constexpr (split_k) {
    if (!split) {
      hipLaunchKernelGGL((layer_kernel<L, P, true>), grid, dim3(kThreads), 0, s, a);
      return;
    }
  }
  hipLaunchKernelGGL((layer_kernel<L, P>), grid, dim3(kThreads), 0, s, a);
  if (split) {
    const long long t = a.M * 512;
    hipLaunchKernelGGL(fc1_reduce_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, a.M, a.part, a.bias,
                       a.acc_scale, reinterpret_cast<float*>(a.out));
  }
}

// item descriptors: the 4 frames of each item's stack
__global__ void item_desc_kernel(long long item_begin, long long n_items, const Seg* __restrict__ segs,
                                 int nsegs, const RootInfo* __restrict__ roots, FrameBases fb,
                                 ItemDesc* __restrict__ out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_items) return;
  const long long item = item_begin + t;
  int lo = 0, hi = nsegs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (segs[mid].item0 <= item) lo = mid; else hi = mid - 1;
  }
  const Seg sg = segs[lo];
  const RootInfo& ri = roots[sg.root];
  const long long j = item - sg.item0;
  ItemDesc d;
  const int m = sg.level;
  // root-local index of the ancestor at each level m, m - 1, .. (through the
  // keep lists of levels cut by a beam)
  long long anc[4];
  anc[3] = j;
  for (int c = 2; c >= 0; --c) {
    const int l = m - 3 + c;          // level of ancestor c
    anc[c] = l >= 1 ? parent_local(ri, fb.keep, l + 1, anc[c + 1]) : -1;
  }
  for (int c = 0; c < 4; ++c) {
    const int l = m - 3 + c;
    if (l >= 1) {
      d.frame[c] = fb.level_frames[l] + (ri.base[l] + anc[c]) * (long long)kFrameBytes;
    } else {
      d.frame[c] = fb.level_frames[0] + ((long long)sg.root * 4 + 3 + l) * (long long)kFrameBytes;
    }
  }
  d.A = sg.A;
  d.q0_root = sg.kind == 2 ? sg.root : -1;
  out[t] = d;
}

template <int P>
void run_qnet(const QnetDev& q, const ItemDesc* desc, long long n, const ChunkGroups& cg, void* ws, float* V,
              float* q0, hipStream_t s, hipEvent_t* ev) {
  typedef typename PT<P>::T T;
  T* x1 = reinterpret_cast<T*>(ws);
  T* x2 = x1 + n * 12800;
  T* x3 = x2 + n * 5184;
  T* h = x3 + n * 3136;
  float* part = reinterpret_cast<float*>(h + n * 512);    // FP32: fc1's K slices
  auto wp = [&](int l) -> const void* {
    return P == P_FP32 ? (const void*)q.w[l] : P == P_BF16 ? (const void*)q.wb[l] : (const void*)q.w8[l];
  };
  // accumulator scales: conv1 sees raw pixels (x 1/255); fp8 undoes both operand scales
  auto accs = [&](int l) {
    float s = (P == P_FP8) ? 1.f / (q.ascale[l] * q.wscale[l]) : 1.f;
    return l == 0 ? s / 255.f : s;
  };
  auto outs = [&](int l) { return (P == P_FP8 && l < 4) ? q.ascale[l + 1] : 1.f; };
  LayerArgs a{};
  a.desc = desc;
  if (ev) (void)hipEventRecord(ev[0], s);
  a.in_s8 = q.ascale[0];
  a.M = n * 400; a.in = nullptr; a.w = wp(0); a.bias = q.b[0]; a.acc_scale = accs(0); a.out_s8 = outs(0); a.out = x1;
  // (the group kernel indexes rows and output rows in 32 bits: chunks of up
  // to 5 M stacks; a larger chunk runs conv1 stack by stack, same results)
  if (cg.n > 0 && n * 400 + kBM < (1LL << 31)) {
    a.M = (long long)cg.n * 400;
    a.groups = cg.groups;
    a.n_groups = cg.n;
    a.item_base = cg.item_base;
    hipLaunchKernelGGL((conv1_groups_kernel<P>), dim3((unsigned)((a.M + kBM - 1) / kBM)), dim3(kThreads), 0, s, a);
  } else {
    run_layer<0, P>(a, s);
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  a.M = n * 81; a.in = x1; a.w = wp(1); a.bias = q.b[1]; a.acc_scale = accs(1); a.out_s8 = outs(1); a.out = x2;
  run_layer<1, P>(a, s);
  if (ev) (void)hipEventRecord(ev[2], s);
  a.M = n * 49; a.in = x2; a.w = wp(2); a.bias = q.b[2]; a.acc_scale = accs(2); a.out_s8 = outs(2); a.out = x3;
  run_layer<2, P>(a, s);
  if (ev) (void)hipEventRecord(ev[3], s);
  a.M = n; a.in = x3; a.w = wp(3); a.bias = q.b[3]; a.acc_scale = accs(3); a.out_s8 = outs(3); a.out = h;
  a.part = part;
  run_layer<3, P>(a, s);
  if (ev) (void)hipEventRecord(ev[4], s);
  a.M = n; a.in = h; a.w = wp(4); a.bias = q.b[4]; a.acc_scale = accs(4); a.out = nullptr; a.V = V; a.q0 = q0;
  run_layer<4, P>(a, s);
  if (ev) (void)hipEventRecord(ev[5], s);
}

// fc1 and fc2 after the fused conv kernel: with `folded` fc2 runs in fc1's
// epilogue (its partial sums take h's place in the workspace), else fc1
// writes h and fc2 + max reads it
template <int P>
void run_fc(const QnetDev& q, const ItemDesc* desc, long long n, const void* x3, void* h, float* V, float* q0,
            hipStream_t s, hipEvent_t ev, bool folded) {
  static_assert(P != P_FP32, "x3 comes from the fused kernel (BF16 / FP8), in stage-major tiles");
  auto accs = [&](int l) { return (P == P_FP8) ? 1.f / (q.ascale[l] * q.wscale[l]) : 1.f; };
  const void* w1 = P == P_BF16 ? (const void*)q.wfb[3] : (const void*)q.wf8[3];
  const void* w2 = P == P_BF16 ? (const void*)q.wb[4] : (const void*)q.w8[4];
  const float out_s8 = P == P_FP8 ? q.ascale[4] : 1.f;
  if (folded) {
    launch_fc12(P, n, x3, w1, q.b[3], accs(3), out_s8, w2, reinterpret_cast<float*>(h), s, ev, q.b[4], accs(4), desc,
                V, q0);
    return;
  }
  launch_fc1_mfma(P, n, x3, w1, q.b[3], accs(3), out_s8, h, s);
  if (ev) (void)hipEventRecord(ev, s);
  LayerArgs a{};
  a.desc = desc;
  a.M = n; a.in = h; a.w = w2; a.bias = q.b[4]; a.acc_scale = accs(4); a.out = nullptr; a.V = V; a.q0 = q0;
  run_layer<4, P>(a, s);
}

__global__ void to_bf16_kernel(const float* __restrict__ s, uint16_t* __restrict__ d, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = f2bf(s[i]);
}
__global__ void to_fp8_kernel(const float* __restrict__ s, uint8_t* __restrict__ d, long long n, float sc) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = f2e4m3(s[i] * sc);
}
__global__ void absmax_kernel(const float* __restrict__ s, long long n, float* out) {
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(s[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(reinterpret_cast<unsigned*>(out), __float_as_uint(m));
}

}  // namespace

void launch_item_desc(long long item_begin, long long n_items, const Seg* segs, int nsegs,
                      const RootInfo* roots, const FrameBases& fb, ItemDesc* out, hipStream_t s) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(item_desc_kernel, dim3((unsigned)((n_items + 255) / 256)), dim3(256), 0, s,
                     item_begin, n_items, segs, nsegs, roots, fb, out);
}

void launch_qnet(int prec, const QnetDev& q, const ItemDesc* desc, long long n, void* ws, float* V,
                 float* q0, hipStream_t s, hipEvent_t* ev) {
  launch_qnet_groups(prec, q, desc, n, ChunkGroups{nullptr, 0, 0}, ws, V, q0, s, ev);
}

void launch_qnet_groups(int prec, const QnetDev& q, const ItemDesc* desc, long long n, const ChunkGroups& cg,
                        void* ws, float* V, float* q0, hipStream_t s, hipEvent_t* ev) {
  if (n <= 0) return;
  if (prec == P_FP32) run_qnet<P_FP32>(q, desc, n, cg, ws, V, q0, s, ev);
  else if (prec == P_BF16) run_qnet<P_BF16>(q, desc, n, cg, ws, V, q0, s, ev);
  else run_qnet<P_FP8>(q, desc, n, cg, ws, V, q0, s, ev);
}

void launch_qnet_fc(int prec, const QnetDev& q, const ItemDesc* desc, long long n, const void* x3, void* h,
                    float* V, float* q0, hipStream_t s, hipEvent_t ev, bool folded) {
  if (n <= 0) return;
  if (prec == P_BF16) run_fc<P_BF16>(q, desc, n, x3, h, V, q0, s, ev, folded);
  else run_fc<P_FP8>(q, desc, n, x3, h, V, q0, s, ev, folded);
}

void launch_convert_bf16(const float* src, uint16_t* dst, long long n, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
}
void launch_convert_fp8(const float* src, uint8_t* dst, long long n, float scale, hipStream_t s) {
  hipLaunchKernelGGL(to_fp8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n, scale);
}
void launch_absmax(const float* src, long long n, float* out, hipStream_t s) {
  long long b = (n + 255) / 256;
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)(b < 1024 ? b : 1024)), dim3(256), 0, s, src, n, out);
}

}  // namespace bcts
