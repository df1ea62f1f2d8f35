// fc1 of the Nature-DQN on the matrix cores: H = ReLU(X W^T + b) with
// X [n][3136] (conv3 output, channels-last) and W [512][3136] (rows re-laid
// out to the same (h, w, c) order), BF16 or OCP e4m3 operands, FP32
// accumulate.  H [n][512] in the operand type feeds fc2, or (the default
// form, FC2) fc2 runs in the epilogue on the same rounded values and H is
// never written.
//
// A workgroup of 8 wavefronts computes a 256 (stacks) x 256 (neurons) tile:
// wave (wm, wn) owns 64 x 128, i.e. 4 x 8 MFMA 16x16x32 fragments, so one
// LDS operand read feeds 4 or 8 MFMAs and each global byte feeds 256 output
// columns.  The product is computed transposed (D[neuron][stack] = W X^T) so
// each lane finishes with 4 consecutive neurons of one stack and stores them
// at once.
//
// K streams through a ring of 5 LDS stages (64 bytes of every tile row per
// stage: 32 K values in BF16, 64 in e4m3), filled by direct global->LDS
// loads (no registers, no LDS store instructions) three stages ahead of the
// MFMAs.  X and W are both stored in stage-major tiles (fc1_tiled_offset):
// the 64-byte slices of a stage's 256 rows form one contiguous 16 KB block,
// so a stage reads two such blocks, where the row-major layout scatters it
// into 512 half cache lines 6,272 bytes apart.  Measured on 748,928 BF16
// stacks, the row-major layout takes 1.25x as long for the loads alone and
// 1.16x for the kernel.  X's rows are padded to a multiple of 256; padding
// rows are read and not stored.
//
// A direct load writes lane l's 16 bytes at slot l of the instruction's 1 KB
// window, so the bank-conflict swizzle is applied on the global side: LDS
// slot (row r, chunk pc) holds the tile's K chunk pc ^ ((r >> 2) & m).  A
// 16-byte LDS read serves each 32-lane half of a wavefront in two cycles, one
// per parity of lane bits 2, 3 and 4, and a cycle is conflict-free when its
// 16 lanes touch 16 distinct 16-byte bank groups (64 banks of 4 bytes); for
// a BF16 operand read (lane = 16 x chunk group + row) m = 2 gives every
// cycle 16 distinct groups, where a plain or m = 3 layout gives 8.  FP8
// operand reads are 8 bytes and take m = 3 (see swz).
// Each stage ends its wavefront's own loads (s_waitcnt vmcnt) before one
// workgroup barrier; the slot a load refills was last read two stages
// earlier, before a barrier every wavefront has passed.
#include "bcts_internal.h"

namespace bcts {
namespace {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;

constexpr int kThreads = 512;
constexpr int kBM = 256, kBN = 256, kK = 3136;
constexpr int kRB = 64;                            // bytes of a tile row per stage
constexpr int kNS = 5;                             // ring stages (5 x 32 KB = the whole LDS)
constexpr int kAhead = kNS - 2;                    // stages in flight ahead of the MFMAs
constexpr int kStageBytes = (kBM + kBN) * kRB;
static_assert(512 / kBN == 2, "the workgroup mapping assumes 2 neuron tiles");
static_assert(kBM == kFc1Rows && kBN == kFc1Rows && kK == kFc1K && kRB == 64, "tiles are the stage-major blocks");
static_assert(kNS * kStageBytes <= 160 * 1024, "the ring must fit the LDS");

__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// wait until at most n of this wavefront's vector-memory operations are outstanding
__device__ __forceinline__ void wait_vm(int n) {
  switch (n) {
    case 0: __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    case 4: __asm__ volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    case 8: __asm__ volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
    default: __asm__ volatile("s_waitcnt vmcnt(12)" ::: "memory"); break;
  }
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
  // 8 consecutive neurons -> one operand (16 bytes)
  __device__ static V pack8(const float (&v)[8], float) {
    unsigned w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      w[k] = __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{v[2 * k], v[2 * k + 1]}, bf16x2));
    return __builtin_bit_cast(V, make_uint4(w[0], w[1], w[2], w[3]));
  }
  __device__ static void st8(void* p, const float (&v)[8], float s8) { *reinterpret_cast<V*>(p) = pack8(v, s8); }
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
  // 8 consecutive neurons, scaled by s8 -> one operand (8 bytes of e4m3)
  __device__ static V pack8(const float (&v)[8], float s8) {
    unsigned w[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      float x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = fminf(fmaxf(v[4 * k + q] * s8, -448.f), 448.f);
      const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(x[0], x[1], 0, false);
      w[k] = (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(x[2], x[3], lo, true);
    }
    return __builtin_bit_cast(V, make_uint2(w[0], w[1]));
  }
  __device__ static void st8(void* p, const float (&v)[8], float s8) { *reinterpret_cast<V*>(p) = pack8(v, s8); }
};

// byte offset of (row r, logical 16-byte chunk c) inside a stage's A or B
// half.  BF16 operand reads are 16 bytes (lane = 16 x chunk group + row):
// chunk c ^ ((r >> 2) & 2).  FP8 operands are read for the K = 128
// instruction: lane group g takes chunks 2 (g & 1) and 2 (g & 1) + 1 of
// stage 2p + (g >> 1), and chunk c ^ ((r >> 3) & 1) gives every cycle of
// those 16-byte reads 16 distinct bank groups (either BF16 form gives 8).
template <int EB> __device__ __forceinline__ int swz_x(int r) { return EB == 1 ? ((r >> 3) & 1) : ((r >> 2) & 2); }
template <int EB> __device__ __forceinline__ int swz(int r, int c) { return r * kRB + ((c ^ swz_x<EB>(r)) << 4); }

template <int P, bool FC2 = false>
__global__ void __launch_bounds__(kThreads, 1)
fc1_kernel(long long n, const unsigned char* __restrict__ X, const unsigned char* __restrict__ W,
           const float* __restrict__ bias, float acc_scale, float out_s8, unsigned char* __restrict__ H,
           const unsigned char* __restrict__ W2, float* __restrict__ part) {
  typedef FT<P> Ft;
  typedef typename Ft::V V;
  constexpr int EB = Ft::EB;
  constexpr int KPS = kRB / EB;                    // K values per stage
  constexpr int NST = kK / KPS;                    // stages: 98 (BF16), 49 (e4m3)
  constexpr int KS = KPS / 32;                     // MFMA K steps per stage
  static_assert(kK % KPS == 0, "K must split into whole stages");
  __shared__ __attribute__((aligned(1024))) unsigned char ring[kNS][kStageBytes];

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
  const int wm = wave >> 1, wn = wave & 1;         // 4 x 2 waves

  // Loads of one stage: 2 instructions for A (X rows) and 2 for B (W rows)
  // per wavefront; instruction q of a half covers LDS slots [64q, 64q + 64)
  // of 16 bytes: slot ps = row ps / 4, physical chunk ps % 4.  In the tiled
  // layout the stage's slice of tile row r starts at stage * 16 KB + 64 r.
  const unsigned char* srcA[2];
  const unsigned char* srcB[2];
  int dst[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int q = wave * 2 + j, ps = q * 64 + lane;
    const int r = ps >> 2, c = (ps & 3) ^ swz_x<EB>(r);
    srcA[j] = X + fc1_tiled_offset(m0 + r, c * 16, EB);
    srcB[j] = W + fc1_tiled_offset(n0 + r, c * 16, EB);
    dst[j] = q * 1024;                              // wave-uniform LDS window
  }
  auto issue = [&](int st) {
    unsigned char* base = ring[st % kNS];
    const long long ko = (long long)st * kFc1StageBytes;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      __builtin_amdgcn_global_load_lds(srcA[j] + ko, (void __attribute__((address_space(3)))*)(base + dst[j]), 16, 0, 0);
      __builtin_amdgcn_global_load_lds(srcB[j] + ko, (void __attribute__((address_space(3)))*)(base + kBM * kRB + dst[j]),
                                       16, 0, 0);
    }
  };

  f32x4 acc[8][4];            // [neuron frag][stack frag]
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  if constexpr (P == P_FP8) {
    // K = 128 instruction over stage pairs (2p, 2p + 1), one barrier per
    // pair; an odd last stage runs on the K = 32 instruction after them.
    // Pair p refills the two slots pair p - 1 read (stages 2p + 3, 2p + 4),
    // after its barrier, which every wavefront passes only once it has
    // finished pair p - 1; stage 2p + 2 is then in flight from pair p - 1.
    typedef __attribute__((ext_vector_type(8))) int v8i;
    typedef __attribute__((ext_vector_type(4))) unsigned u32x4;
    auto ld32 = [](const unsigned char* base, int row, int c) {
      const u32x4 lo = *reinterpret_cast<const u32x4*>(base + swz<EB>(row, c));
      const u32x4 hi = *reinterpret_cast<const u32x4*>(base + swz<EB>(row, c + 1));
      return v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
    };
    static_assert(kAhead == 3 && kNS == 5, "the pair schedule assumes 5 slots, 3 stages issued ahead");
#pragma unroll
    for (int st = 0; st < kAhead; ++st) issue(st);
    for (int pp = 0; pp < NST / 2; ++pp) {
      wait_vm(2 * pp + 2 < NST ? 4 : 0);            // stage 2p + 2 may stay in flight
      lds_barrier();
      if (2 * pp + 3 < NST) issue(2 * pp + 3);
      if (2 * pp + 4 < NST) issue(2 * pp + 4);
      // this lane's K chunk: stage 2p + (g >> 1), bytes 32 (g & 1) .. +31
      const unsigned char* As = ring[(2 * pp + (g >> 1)) % kNS];
      const unsigned char* Bs = As + kBM * kRB;
      const int c0 = 2 * (g & 1);
      // neuron fragment i + 1's operand is read before fragment i's MFMAs
      // (two register sets; scheduling barriers keep that order, else the
      // compiler hoists all eight reads and runs out of registers)
      v8i xv[4], wv[2];
#pragma unroll
      for (int j = 0; j < 4; ++j) xv[j] = ld32(As, wm * 64 + j * 16 + r16, c0);
      wv[0] = ld32(Bs, wn * 128 + r16, c0);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (i + 1 < 8) wv[(i + 1) & 1] = ld32(Bs, wn * 128 + (i + 1) * 16 + r16, c0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(wv[i & 1], xv[j], acc[i][j], 0, 0, 0, 127, 0,
                                                                        127);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if constexpr (NST & 1) {
      wait_vm(0);
      lds_barrier();
      const unsigned char* As = ring[(NST - 1) % kNS];
      const unsigned char* Bs = As + kBM * kRB;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int kb = ks * 32 * EB + 8 * g * EB;
        const int c = kb >> 4, cb = kb & 15;
        V xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[j] = *reinterpret_cast<const V*>(As + swz<EB>(wm * 64 + j * 16 + r16, c) + cb);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const V wv = *reinterpret_cast<const V*>(Bs + swz<EB>(wn * 128 + i * 16 + r16, c) + cb);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = Ft::mma(wv, xv[j], acc[i][j]);
        }
      }
    }
  } else {
#pragma unroll
    for (int st = 0; st < kAhead; ++st) issue(st);
    for (int st = 0; st < NST; ++st) {
      if (st + kAhead < NST) issue(st + kAhead);
      const int later = (NST - 1 - st) < kAhead ? (NST - 1 - st) : kAhead;   // stages issued after st
      wait_vm(4 * later);
      lds_barrier();
      const unsigned char* As = ring[st % kNS];
      const unsigned char* Bs = As + kBM * kRB;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        // this lane's 8 K values of step ks: byte 32 * ks * EB / ... within the row
        const int kb = ks * 32 * EB + 8 * g * EB;        // byte offset in the row's 64 bytes
        const int c = kb >> 4, cb = kb & 15;
        V xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) xv[j] = *reinterpret_cast<const V*>(As + swz<EB>(wm * 64 + j * 16 + r16, c) + cb);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const V wv = *reinterpret_cast<const V*>(Bs + swz<EB>(wn * 128 + i * 16 + r16, c) + cb);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = Ft::mma(wv, xv[j], acc[i][j]);
        }
      }
    }
  }

  // epilogue: the weight rows are paired (fc1_weight_tiles_kernel), so
  // fragments 2k and 2k + 1 give the lane neurons n0 + wn*128 + 32k + 8g
  // + 0..7 of stack m0 + wm*64 + 16j + r16: one 16-byte (BF16) or 8-byte
  // (FP8) store
  if constexpr (FC2) {
    // fc2 on the wavefront's 128 neurons, 4 K steps of 32: A = fc2's weight
    // rows (actions 16 af + r16, K values 8g .. 8g + 7 of the step), B = the
    // lane's 8 neurons of stack 16 j + r16 in the operand type, the values h
    // would hold: the same operands as fc2 on h, without h
    f32x4 q2[2][4];
#pragma unroll
    for (int af = 0; af < 2; ++af)
#pragma unroll
      for (int j = 0; j < 4; ++j) q2[af][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int nb = n0 + wn * 128 + 32 * k + 8 * g;
      float b[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) b[e] = bias[nb + e];
      V w2[2];
#pragma unroll
      for (int af = 0; af < 2; ++af)
        w2[af] = *reinterpret_cast<const V*>(W2 + ((size_t)(af * 16 + r16) * 512 + nb) * EB);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float v[8];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int q = 0; q < 4; ++q) v[4 * h + q] = fmaxf(acc[2 * k + h][j][q] * acc_scale + b[4 * h + q], 0.f);
        const V hv = Ft::pack8(v, out_s8);
#pragma unroll
        for (int af = 0; af < 2; ++af) q2[af][j] = Ft::mma(w2[af], hv, q2[af][j]);
      }
    }
    // the tile's two neuron halves (wn = 0, 1) added in that order, through
    // the ring (every wavefront has finished reading it at the barrier):
    // element e of lane l of wave (wm, 1) at [e][wm][l]
    float* xq = reinterpret_cast<float*>(&ring[0][0]);
    lds_barrier();
    if (wn == 1) {
#pragma unroll
      for (int af = 0; af < 2; ++af)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) xq[(((af * 4 + j) * 4 + q) * 4 + wm) * 64 + lane] = q2[af][j][q];
    }
    lds_barrier();
    if (wn == 0) {
      // part[half][stack][32]: this tile's sum over its 256 neurons; lane
      // holds actions 16 af + 4g + q of stack m0 + wm*64 + 16j + r16
      float* P2 = part + (size_t)(slot & 1) * n * 32;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long long m = m0 + wm * 64 + 16 * j + r16;
#pragma unroll
        for (int af = 0; af < 2; ++af) {
          f32x4 t;
#pragma unroll
          for (int q = 0; q < 4; ++q) t[q] = q2[af][j][q] + xq[(((af * 4 + j) * 4 + q) * 4 + wm) * 64 + lane];
          if (m < n) *reinterpret_cast<f32x4*>(P2 + m * 32 + 16 * af + 4 * g) = t;
        }
      }
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int nb = n0 + wn * 128 + 32 * k + 8 * g;
    float b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = bias[nb + e];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long m = m0 + wm * 64 + 16 * j + r16;
      if (m < n) {
        float v[8];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int q = 0; q < 4; ++q) v[4 * h + q] = fmaxf(acc[2 * k + h][j][q] * acc_scale + b[4 * h + q], 0.f);
        Ft::st8(H + (m * 512 + nb) * EB, v, out_s8);
      }
    }
  }
}

// fc2 after fc1_kernel<P, true>: Q[a] = (part_0[a] + part_1[a]) * scale
// + b[a] (the two neuron halves in order); V = max over the stack's A
// actions; a root item's q0 row.  Two stacks per wavefront, lane = action.
__global__ void __launch_bounds__(256) fc2_sum_kernel(long long n, const float* __restrict__ part,
                                                      const float* __restrict__ bias, float scale,
                                                      const ItemDesc* __restrict__ desc, float* __restrict__ V,
                                                      float* __restrict__ q0) {
  const long long m = (long long)blockIdx.x * 8 + (threadIdx.x >> 5);
  const int a = threadIdx.x & 31;
  const bool in = m < n;
  const long long mm = in ? m : 0;
  const float qv = fmaf(part[mm * 32 + a] + part[(n + mm) * 32 + a], scale, a < kMaxA ? bias[a] : 0.f);
  const ItemDesc d = desc[mm];
  float v = a < d.A ? qv : -INFINITY;
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if (!in) return;
  if (a == 0) V[m] = v;
  if (d.q0_root >= 0 && a < kMaxA) q0[(long long)d.q0_root * kMaxA + a] = qv;
}

// one thread per 16 bytes of W[N][K]
__global__ void fc1_weight_tiles_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst,
                                        int N, int K, int eb) {
  const long long per_row = (long long)K * eb / 16;
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= N * per_row) return;
  const long long r = u / per_row;
  const int kb = (int)(u % per_row) * 16;
  // row rho of fragment 2k + h (tile rows 32k .. 32k + 31) holds neuron
  // 32k + 8 (rho / 4) + 4h + rho % 4
  const int w = (int)(r & 31), h = w >> 4, rho = w & 15;
  const long long sr = (r & ~31LL) + 8 * (rho >> 2) + 4 * h + (rho & 3);
  *reinterpret_cast<uint4*>(dst + fc1_tiled_offset(r, kb, eb)) =
      *reinterpret_cast<const uint4*>(src + sr * K * eb + kb);
}

}  // namespace

void launch_fc1_weight_tiles(const void* src, void* dst, int N, int K, int eb, hipStream_t s) {
  const long long units = (long long)N * K * eb / 16;
  hipLaunchKernelGGL(fc1_weight_tiles_kernel, dim3((unsigned)((units + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const unsigned char*>(src), reinterpret_cast<unsigned char*>(dst), N, K, eb);
}

void launch_fc1_mfma(int prec, long long n, const void* x3, const void* w, const float* bias, float acc_scale,
                     float out_s8, void* h, hipStream_t s) {
  if (n <= 0) return;
  const long long mtiles = ((n + kBM - 1) / kBM + 7) / 8 * 8;
  dim3 grid((unsigned)(mtiles * (512 / kBN))), block(kThreads);
  const unsigned char* X = reinterpret_cast<const unsigned char*>(x3);
  const unsigned char* Wp = reinterpret_cast<const unsigned char*>(w);
  unsigned char* H = reinterpret_cast<unsigned char*>(h);
  if (prec == P_BF16)
    hipLaunchKernelGGL((fc1_kernel<P_BF16>), grid, block, 0, s, n, X, Wp, bias, acc_scale, out_s8, H, nullptr, nullptr);
  else
    hipLaunchKernelGGL((fc1_kernel<P_FP8>), grid, block, 0, s, n, X, Wp, bias, acc_scale, out_s8, H, nullptr, nullptr);
}

void launch_fc12(int prec, long long n, const void* x3, const void* w1, const float* b1, float scale1, float out_s8,
                 const void* w2, float* part, hipStream_t s, hipEvent_t ev_after_fc1, const float* b2, float scale2,
                 const ItemDesc* desc, float* V, float* q0) {
  if (n <= 0) return;
  const long long mtiles = ((n + kBM - 1) / kBM + 7) / 8 * 8;
  dim3 grid((unsigned)(mtiles * (512 / kBN))), block(kThreads);
  const unsigned char* X = reinterpret_cast<const unsigned char*>(x3);
  const unsigned char* W1 = reinterpret_cast<const unsigned char*>(w1);
  const unsigned char* W2 = reinterpret_cast<const unsigned char*>(w2);
  if (prec == P_BF16)
    hipLaunchKernelGGL((fc1_kernel<P_BF16, true>), grid, block, 0, s, n, X, W1, b1, scale1, out_s8, nullptr, W2, part);
  else
    hipLaunchKernelGGL((fc1_kernel<P_FP8, true>), grid, block, 0, s, n, X, W1, b1, scale1, out_s8, nullptr, W2, part);
  if (ev_after_fc1) (void)hipEventRecord(ev_after_fc1, s);
  hipLaunchKernelGGL(fc2_sum_kernel, dim3((unsigned)((n + 7) / 8)), dim3(256), 0, s, n, part, b2, scale2, desc, V, q0);
}

}  // namespace bcts
