// Level expansion of Batch-BFS (Alg. 1, loop body): every node of level k-1
// is stepped for all A actions at once.  Node j*A + a of level k is child a
// of node j; per node the kernel writes the moved positions, the rendered
// 84x84 uint8 frame, the integer reward and the discounted return
// ret_k = ret_{k-1} + gamma^(k-1) r  (accumulated in FP32).
//
// The stack is not replicated: a frame is written once, at the node that
// renders it; Q-network inputs read the 4 ancestor frames in place.
//
// Work split: a 256-thread workgroup takes 8 nodes at a time.
//   1. one thread per node: find the root, read the parent, move, score;
//   2. per (node, row): the row's coverage as two 84-bit masks (value 255
//      from sprite 0, 128 from the others), kept in LDS;
//   3. per (node, 16-byte chunk of the flat frame): expand the masks to
//      bytes and store 16 B -- consecutive threads write consecutive chunks,
//      so every wavefront store covers 1 KiB of contiguous HBM.
#include "bcts_internal.h"

namespace bcts {
namespace {

constexpr int kNB = 8;                       // nodes per workgroup iteration
constexpr int kChunks = kFrameBytes / 16;    // 441 16-byte chunks per frame
constexpr int kThreads = 256;

struct RowMask {                             // bits 0..83 of one frame row
  unsigned long long lo255, lo128;           // bits 0..63
  unsigned hi255, hi128;                     // bits 64..83
};

__device__ __forceinline__ int wrap84(int v) {
  v %= kFrame;
  return v < 0 ? v + kFrame : v;
}

// set bits [a, b) (0 <= a < b <= 84) of an 84-bit row
__device__ __forceinline__ void set_bits(unsigned long long& lo, unsigned& hi, int a, int b) {
  if (a < 64) {
    int e = b < 64 ? b : 64;
    unsigned long long m = (e - a == 64) ? ~0ull : (((1ull << (e - a)) - 1ull) << a);
    lo |= m;
  }
  if (b > 64) {
    int s = a > 64 ? a : 64;
    hi |= ((1u << (b - s)) - 1u) << (s - 64);
  }
}

// columns covered by a square anchored at x: [x, x+6) modulo 84
__device__ __forceinline__ void col_mask(int x, unsigned long long& lo, unsigned& hi) {
  lo = 0ull;
  hi = 0u;
  if (x + 6 <= kFrame) {
    set_bits(lo, hi, x, x + 6);
  } else {
    set_bits(lo, hi, x, kFrame);
    set_bits(lo, hi, 0, x + 6 - kFrame);
  }
}

// `len` (<= 16) bits of an 84-bit row starting at bit `st`
__device__ __forceinline__ unsigned take_bits(unsigned long long lo, unsigned hi, int st, int len) {
  unsigned long long v;
  if (st >= 64) {
    v = (unsigned long long)(hi >> (st - 64));
  } else if (st == 0) {
    v = lo;
  } else {
    v = (lo >> st) | ((unsigned long long)hi << (64 - st));
  }
  return (unsigned)(v & ((1ull << len) - 1ull));
}

// 4 mask bits -> 4 bytes of 0/1
__device__ __forceinline__ unsigned spread4(unsigned nib) {
  return (nib * 0x00204081u) & 0x01010101u;
}

__device__ __forceinline__ unsigned pix4(unsigned m255, unsigned m128) {
  unsigned e255 = spread4(m255 & 15u), e128 = spread4(m128 & 15u);
  return e255 * 255u | (e128 & ~(e255 * 255u)) * 128u;
}

__device__ __forceinline__ int find_root(const LevelRoots& lr, long long node) {
  int lo = 0, hi = lr.cnt - 1;
  while (lo < hi) {                           // last entry with start <= node
    int mid = (lo + hi + 1) >> 1;
    if (lr.start[mid] <= node) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Beam cut of level k, one workgroup per (root, root action a0): a0's
// block of the level (c contiguous root-local nodes, c <= A * beam) is ranked
// by return, descending, ties to the lower index (rank of i = number of j
// with ret_j > ret_i, or ret_j == ret_i and j < i: exact, order-free); the
// nodes of rank < beam are written ascending to the keep list.
constexpr int kPruneThreads = 256;
constexpr int kMaxBlock = kMaxA * kMaxBeam;

__global__ void __launch_bounds__(kPruneThreads)
prune_kernel(int k, LevelRoots lr, const RootInfo* __restrict__ roots, const float* __restrict__ ret_k,
             int* __restrict__ keep_k, int beam) {
  __shared__ float v[kMaxBlock];
  __shared__ int kept[kMaxBlock];
  const int r = lr.root[blockIdx.x / kMaxA], a0 = blockIdx.x % kMaxA;
  const RootInfo& ri = roots[r];
  if (a0 >= ri.A || ri.kbase[k] < 0) return;
  const int c = (int)(ri.lcnt[k] / ri.A);          // block size, <= A * beam
  const long long first = ri.base[k] + (long long)a0 * c;
  for (int i = threadIdx.x; i < c; i += kPruneThreads) v[i] = ret_k[first + i];
  __syncthreads();
  for (int i = threadIdx.x; i < c; i += kPruneThreads) {
    const float x = v[i];
    int rank = 0;
    for (int j = 0; j < c; ++j) rank += (v[j] > x || (v[j] == x && j < i)) ? 1 : 0;
    kept[i] = rank < beam ? 1 : 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < c; i += kPruneThreads) {
    if (!kept[i]) continue;
    int pos = 0;
    for (int j = 0; j < i; ++j) pos += kept[j];
    keep_k[ri.kbase[k] + (long long)a0 * beam + pos] = a0 * c + i;
  }
}

__global__ void __launch_bounds__(kThreads)
expand_kernel(int k, long long n_nodes, LevelRoots lr, const RootInfo* __restrict__ roots,
              const int* __restrict__ root_pos, const uint8_t* __restrict__ prev_pos,
              const float* __restrict__ prev_ret, const int* __restrict__ prev_keep, EnvTables env, float gamma_pow,
              uint8_t* __restrict__ pos, uint8_t* __restrict__ frames, float* __restrict__ ret,
              uint8_t* __restrict__ rew_out) {
  __shared__ int s_pos[kNB][kSprites][2];
  __shared__ RowMask s_rows[kNB][kFrame];
  __shared__ unsigned long long s_clo[kNB][kSprites];
  __shared__ unsigned s_chi[kNB][kSprites];

  const int tid = threadIdx.x;
  for (long long g0 = (long long)blockIdx.x * kNB; g0 < n_nodes; g0 += (long long)gridDim.x * kNB) {
    const int nb = (int)((n_nodes - g0) < kNB ? (n_nodes - g0) : kNB);

    // 1. move and score, one thread per node
    if (tid < nb) {
      const long long node = g0 + tid;
      const int ri = find_root(lr, node);
      const int r = lr.root[ri];
      const long long j = node - lr.start[ri];
      const int A = roots[r].A;
      const int a = (int)(j % A);
      const long long pj = roots[r].kbase[k - 1] >= 0 && k > 1 ? (long long)prev_keep[roots[r].kbase[k - 1] + j / A]
                                                              : j / A;
      int p[kSprites][2];
      float pret = 0.f;
      if (k == 1) {
        const int* rp = root_pos + (long long)r * kSprites * 2;
        for (int i = 0; i < kSprites; ++i) {
          p[i][0] = wrap84(rp[2 * i]);
          p[i][1] = wrap84(rp[2 * i + 1]);
        }
      } else {
        const long long pn = roots[r].base[k - 1] + pj;
        const uint4 v = *reinterpret_cast<const uint4*>(prev_pos + pn * 16);
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
        for (int i = 0; i < kSprites; ++i) {
          const unsigned word = w[i >> 1] >> ((i & 1) * 16);
          p[i][0] = word & 255u;
          p[i][1] = (word >> 8) & 255u;
        }
        pret = prev_ret[pn];
      }
      p[0][0] = wrap84(p[0][0] + env.delta[a][0]);
      p[0][1] = wrap84(p[0][1] + env.delta[a][1]);
      for (int i = 1; i < kSprites; ++i) {
        p[i][0] = wrap84(p[i][0] + env.vel[i - 1][0]);
        p[i][1] = wrap84(p[i][1] + env.vel[i - 1][1]);
      }
      int rew = 0;
      for (int i = 1; i < kSprites; ++i) {
        int dx = wrap84(p[0][0] - p[i][0]), dy = wrap84(p[0][1] - p[i][1]);
        dx = dx < kFrame - dx ? dx : kFrame - dx;
        dy = dy < kFrame - dy ? dy : kFrame - dy;
        rew += (dx < 6 && dy < 6) ? 1 : 0;
      }
      unsigned w[4];
      for (int q = 0; q < 4; ++q)
        w[q] = (unsigned)p[2 * q][0] | ((unsigned)p[2 * q][1] << 8) |
               ((unsigned)p[2 * q + 1][0] << 16) | ((unsigned)p[2 * q + 1][1] << 24);
      *reinterpret_cast<uint4*>(pos + node * 16) = make_uint4(w[0], w[1], w[2], w[3]);
      ret[node] = fmaf(gamma_pow, (float)rew, pret);   // one rounding (a beam ranks these)
      rew_out[node] = (uint8_t)rew;
      for (int i = 0; i < kSprites; ++i) {
        s_pos[tid][i][0] = p[i][0];
        s_pos[tid][i][1] = p[i][1];
      }
    }
    __syncthreads();
    if (tid < nb * kSprites) {
      const int b = tid / kSprites, i = tid % kSprites;
      col_mask(s_pos[b][i][0], s_clo[b][i], s_chi[b][i]);
    }
    __syncthreads();

    // 2. row masks
    for (int t = tid; t < nb * kFrame; t += kThreads) {
      const int b = t / kFrame, y = t % kFrame;
      RowMask m = {0ull, 0ull, 0u, 0u};
      for (int i = 0; i < kSprites; ++i) {
        if (wrap84(y - s_pos[b][i][1]) < 6) {
          if (i == 0) { m.lo255 |= s_clo[b][i]; m.hi255 |= s_chi[b][i]; }
          else        { m.lo128 |= s_clo[b][i]; m.hi128 |= s_chi[b][i]; }
        }
      }
      s_rows[b][y] = m;
    }
    __syncthreads();

    // 3. 16-byte chunks of the frames
    for (int t = tid; t < nb * kChunks; t += kThreads) {
      const int b = t / kChunks, c = t % kChunks;
      const int o = c * 16, y0 = o / kFrame, x0 = o % kFrame;
      const int len0 = (kFrame - x0) < 16 ? (kFrame - x0) : 16;
      const RowMask& r0 = s_rows[b][y0];
      unsigned m255 = take_bits(r0.lo255, r0.hi255, x0, len0);
      unsigned m128 = take_bits(r0.lo128, r0.hi128, x0, len0);
      if (len0 < 16) {
        const RowMask& r1 = s_rows[b][y0 + 1];
        m255 |= take_bits(r1.lo255, r1.hi255, 0, 16 - len0) << len0;
        m128 |= take_bits(r1.lo128, r1.hi128, 0, 16 - len0) << len0;
      }
      uint4 v;
      v.x = pix4(m255, m128);
      v.y = pix4(m255 >> 4, m128 >> 4);
      v.z = pix4(m255 >> 8, m128 >> 8);
      v.w = pix4(m255 >> 12, m128 >> 12);
      *reinterpret_cast<uint4*>(frames + (g0 + b) * kFrameBytes + o) = v;
    }
    __syncthreads();
  }
}

}  // namespace

void launch_expand(int k, long long n_nodes, LevelRoots lr, const RootInfo* roots,
                   const int* root_pos, const uint8_t* prev_pos, const float* prev_ret, const int* prev_keep,
                   const EnvTables& env, float gamma_pow, uint8_t* pos, uint8_t* frames,
                   float* ret, uint8_t* rew, hipStream_t s) {
  if (n_nodes <= 0) return;
  // One workgroup per group of kNB nodes (the loop covers grids capped at
  // 2^20 workgroups).  Measured on the 1.49M-node level of the headline
  // shape: capping the grid at 65,536 workgroups that loop over several
  // groups, or marking the frame stores non-temporal, each slows the
  // level's HBM write stream (the three levels take 8% longer with both).
  long long groups = (n_nodes + kNB - 1) / kNB;
  int grid = (int)(groups < (1 << 20) ? groups : (1 << 20));
  hipLaunchKernelGGL(expand_kernel, dim3(grid), dim3(kThreads), 0, s, k, n_nodes, lr, roots,
                     root_pos, prev_pos, prev_ret, prev_keep, env, gamma_pow, pos, frames, ret, rew);
}

void launch_prune(int k, int n_level_roots, LevelRoots lr, const RootInfo* roots, const float* ret_k, int* keep_k,
                  int beam, hipStream_t s) {
  if (n_level_roots <= 0) return;
  hipLaunchKernelGGL(prune_kernel, dim3((unsigned)n_level_roots * kMaxA), dim3(kPruneThreads), 0, s, k, lr, roots,
                     ret_k, keep_k, beam);
}

}  // namespace bcts
