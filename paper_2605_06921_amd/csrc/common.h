// Shared device helpers of libmqo (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mqo {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): per round two 64x64
// multiplications, output (hi1^c1^k0, lo1, hi0^c3^k1, lo0), key bumped by
// the Weyl constants between rounds.
// Stream layout: key = (seed, purpose), counter = (v >> 3, t, round, 0);
// vertex v takes 32-bit lane v & 7 (word (v & 7) >> 1, low half if even).
// ---------------------------------------------------------------------------
enum : uint64_t {
  PURPOSE_INIT = 1,
  PURPOSE_RESET = 2,
  PURPOSE_LS = 3,
  PURPOSE_NOISE = 4,
  PURPOSE_SWAP = 5,
  PURPOSE_TOY_RESET = 6,
  PURPOSE_TOY_START = 7,
  PURPOSE_POOL = 8
};

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0;
    const uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// The 8 uint32 draws of vertices 8*vb .. 8*vb+7.
__device__ __forceinline__ void philox_block8(uint32_t out[8], uint64_t seed, uint64_t purpose,
                                              uint64_t traj, uint64_t round, uint64_t vb) {
  uint64_t c[4] = {vb, traj, round, 0};
  philox4x64_10(c, seed, purpose);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    out[2 * i] = (uint32_t)c[i];
    out[2 * i + 1] = (uint32_t)(c[i] >> 32);
  }
}

__device__ __forceinline__ uint32_t philox_vertex(uint64_t seed, uint64_t purpose, uint64_t traj,
                                                  uint64_t round, uint64_t v) {
  uint64_t c[4] = {v >> 3, traj, round, 0};
  philox4x64_10(c, seed, purpose);
  const uint32_t lane = (uint32_t)(v & 7);
  const uint64_t w = lane < 2 ? c[0] : lane < 4 ? c[1] : lane < 6 ? c[2] : c[3];
  return (uint32_t)(w >> (32 * (lane & 1)));
}

// 24 random bits as an exact float in [0, 1).
__device__ __forceinline__ float unit_f32(uint32_t u) { return (float)(u >> 8) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------------------
// The objective as ascended: MIS g = 1 - gamma*acc on [0,1];
// MaxCut g = (-lambda) - 2*acc on [-1,1].  One rounding per operation
// (built with -ffp-contract=off).
// ---------------------------------------------------------------------------
template <bool MAXCUT>
__device__ __forceinline__ float grad_from_sum(float acc, float param) {
  if (MAXCUT) {
    // 2 * acc is exact, so the fused form rounds (-lambda) - 2 * acc once,
    // exactly as the two-operation form does
    return fmaf(-2.0f, acc, -param);
  } else {
    const float t = param * acc;
    return 1.0f - t;
  }
}

// The continuous objective of a PGA step: MIS h (Eq. (3)) or one of the
// MaxCut formulations of Sec. 3 (the algorithms use f_B).
enum : int { OBJ_H = 0, OBJ_FB = 1, OBJ_FL = 2, OBJ_FP = 3, OBJ_FA = 4 };

// Gradient at x_v from acc = (A x)_v and the weighted degree W_v (used by
// f_L, f_P), one float32 rounding per operation in the order written:
// f_L 0.5 (W x - acc) (Eq. (4)), f_P 2 ((W x - acc) + lambda x) (Eq. (5)),
// f_A -2 acc (Eq. (6)); h and f_B as grad_from_sum.
template <int OBJ>
__device__ __forceinline__ float grad_of(float acc, float x, float W, float param);

template <bool MAXCUT>
__device__ __forceinline__ float box_lo() { return MAXCUT ? -1.0f : 0.0f; }
__device__ __forceinline__ float box_hi() { return 1.0f; }

template <bool MAXCUT>
__device__ __forceinline__ float clip_box(float y) {
  return fminf(fmaxf(y, box_lo<MAXCUT>()), box_hi());
}

template <int OBJ>
__device__ __forceinline__ float grad_of(float acc, float x, float W, float param) {
  if constexpr (OBJ == OBJ_H || OBJ == OBJ_FB) {
    return grad_from_sum<OBJ == OBJ_FB>(acc, param);
  } else if constexpr (OBJ == OBJ_FA) {
    return -2.0f * acc;
  } else {
    const float t1 = W * x;
    const float t2 = t1 - acc;
    if constexpr (OBJ == OBJ_FL) {
      return 0.5f * t2;
    } else {
      const float t3 = param * x;
      const float t4 = t2 + t3;
      return 2.0f * t4;
    }
  }
}

// Threshold rounding of Sec. 3: MIS x > 0.5 -> 1 else 0; MaxCut x > 0 -> +1 else -1.
template <bool MAXCUT>
__device__ __forceinline__ int8_t round_x(float x) {
  if (MAXCUT) return x > 0.0f ? (int8_t)1 : (int8_t)-1;
  return x > 0.5f ? (int8_t)1 : (int8_t)0;
}

// Positive-gain test of the 1-flip search and the first key component:
// MaxCut gain s_v t_v > 0 (k1 = gain); MIS removal of v in I with m_v >= 1
// (k1 = m_v) or addition of v not in I with m_v = 0 (k1 = 0).
template <bool MAXCUT>
__device__ __forceinline__ bool ls_candidate_t(int32_t z, int32_t nb, int32_t &k1) {
  if (MAXCUT) {
    k1 = z * nb;
    return k1 > 0;
  }
  if (z) {
    k1 = nb;
    return nb >= 1;
  }
  k1 = 0;
  return nb == 0;
}

// Lexicographic local-search key (k1, prio, -v): true iff (k1a,pa,va) beats (k1b,pb,vb).
__device__ __forceinline__ bool key_beats(int32_t k1a, uint32_t pa, int64_t va, int32_t k1b, uint32_t pb,
                                          int64_t vb) {
  if (k1a != k1b) return k1a > k1b;
  if (pa != pb) return pa > pb;
  return va < vb;
}

// Executed by one whole wavefront (64 lanes, threadIdx.x & 63 = lane):
// hist[0..255] counts keys per digit; finds the digit bin holding the
// krem-th smallest key (1-based, krem <= total), the count of keys in the
// bins before it and the count in it.  Lane l owns bins 4l .. 4l+3.
__device__ __forceinline__ void wave_select_digit(const uint32_t *hist, uint32_t krem, uint32_t &digit,
                                                  uint32_t &before, uint32_t &at) {
  const int lane = threadIdx.x & 63;
  uint32_t h[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) h[i] = hist[lane * 4 + i];
  const uint32_t own = h[0] + h[1] + h[2] + h[3];
  uint32_t incl = own;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  const uint32_t excl = incl - own;
  const unsigned long long mask = __ballot(excl < krem && krem <= incl);
  const int src = mask ? __builtin_ctzll(mask) : 63;
  // inside the lane: the one bin where the running count first reaches krem
  uint32_t d = lane * 4 + 3, b = excl, a = h[3], run = excl;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (run < krem && krem <= run + h[i]) {
      d = lane * 4 + i;
      b = run;
      a = h[i];
    }
    run += h[i];
  }
  digit = __shfl(d, src, 64);
  before = __shfl(b, src, 64);
  at = __shfl(a, src, 64);
}

// Sum of v over the lanes of the wavefront that share lane % width (width a
// power of two <= 64); the result is valid in lanes 0 .. width-1.  Every
// lane must call it.
__device__ __forceinline__ long long wave_sum_stride(long long v, int width) {
  for (int off = 32; off >= width; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// One graph of a batch as the kernels see it.
struct GraphView {
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const int32_t *weight;  // nullptr = unit
  int64_t lo;             // first global row of the graph
  int64_t n;              // rows of the graph
  const int32_t *hubs;    // global ids of the rows of degree > hub_deg, ascending
  int32_t nhub;           // 0 = no hub list
  int32_t hub_deg;
  int32_t pairs;          // 1: near-regular graph, lane groups take rows in pairs
  int32_t xcd_local;      // 1: rows close in the vertex order share neighbours (one row range per XCD)
};

// Row x column mapping: W lanes per row (power of two <= 64), each lane
// owning VEC consecutive columns; blockIdx.y walks column chunks.
struct RowMap {
  int64_t row;
  int32_t col;
  bool active;
};

// Lane group of 2^lanes_log2 lanes per row; bx is the workgroup's index
// among the row workgroups of the launch.
template <int VEC>
__device__ __forceinline__ RowMap map_rows(int64_t nrows, int32_t ncols, int32_t lanes_log2, int64_t bx) {
  RowMap m;
  const int32_t lanes = 1 << lanes_log2;
  const int32_t rows_per_block = blockDim.x >> lanes_log2;
  m.row = bx * rows_per_block + (threadIdx.x >> lanes_log2);
  m.col = (int32_t)(blockIdx.y * lanes + (threadIdx.x & (lanes - 1))) * VEC;
  m.active = m.row < nrows && m.col < ncols;
  return m;
}

template <int VEC>
__device__ __forceinline__ RowMap map_rows(int64_t nrows, int32_t ncols, int32_t lanes_log2) {
  return map_rows<VEC>(nrows, ncols, lanes_log2, (int64_t)blockIdx.x);
}

}  // namespace mqo
