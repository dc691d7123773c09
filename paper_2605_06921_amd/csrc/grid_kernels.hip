// Grid-wide kernels of libmqo: one graph per launch, rows of the graph x
// columns (trajectories) of the batch.  Used by the batched and plain plans,
// by the building-block entry points and by differentiation.
//
// Element (v, c) of an [n][ld] array lives at v * ld + c with v the GLOBAL
// row; random draws use the local index v - lo and the trajectory id
// traj0 + c.
#include <algorithm>
#include <climits>

#include "common.h"
#include "kernels.h"

namespace mqo {

static inline int lanes_log2_for(int cols) {
  int w = 1, l = 0;
  while (w < cols && w < 64) {
    w <<= 1;
    ++l;
  }
  return l;
}

static inline dim3 grid_rows(int64_t nrows, int ncols, int lanes_log2, int vec, int threads) {
  const int lanes = 1 << lanes_log2;
  const int64_t rpb = threads >> lanes_log2;
  const int64_t gx = (nrows + rpb - 1) / rpb;
  const int gy = (ncols + lanes * vec - 1) / (lanes * vec);
  return dim3((unsigned)(gx > 0 ? gx : 1), (unsigned)(gy > 0 ? gy : 1), 1);
}

// Workgroups are handed to the 8 XCDs (each with its own L2) round-robin in
// launch order, linear id x + y gridDim.x.  On graphs with locality (grids,
// tori, banded orders: the graph's local_rows hint) the sparse-product
// kernels renumber them so that each XCD runs one contiguous range of the
// (row block, column slice) space: rows close in the vertex order, which
// gather many of the same rows of X, then share one L2 instead of fetching
// those rows once per XCD.  Elsewhere the launch order stands: it spreads
// rows that are heavy together (the early vertices of preferential
// attachment) over all XCDs.  A bijection of the launch, so every result is
// unchanged.
struct Blk {
  int64_t x;
  int32_t y;
};

__device__ __forceinline__ Blk xcd_blk(bool local) {
  if (!local) return Blk{blockIdx.x, (int32_t)blockIdx.y};
  const int64_t gx = gridDim.x, nb = gx * gridDim.y;
  const int64_t b = blockIdx.x + (int64_t)blockIdx.y * gx;
  const int64_t q = nb >> 3, r = nb & 7, xcd = b & 7, j = b >> 3;
  const int64_t l = xcd * q + (xcd < r ? xcd : r) + j;
  return Blk{l % gx, (int32_t)(l / gx)};
}

// ---------------------------------------------------------------------------
// initialisation
// ---------------------------------------------------------------------------
// start: index of the fresh start (the round field of the Philox counter)
template <bool MAXCUT>
__global__ __launch_bounds__(256) void k_init_uniform(float *__restrict__ X, int64_t lo, int64_t n, int32_t ncols,
                                                      int32_t ld, uint64_t seed, uint64_t traj0, uint64_t start) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nvb = (n + 7) >> 3;
  if (idx >= nvb * ncols) return;
  const int32_t c = (int32_t)(idx % ncols);
  const int64_t vb = idx / ncols;
  uint32_t r[8];
  philox_block8(r, seed, PURPOSE_INIT, traj0 + c, start, (uint64_t)vb);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t v = vb * 8 + i;
    if (v < n) {
      const float u = unit_f32(r[i]);
      float x;
      if (MAXCUT) {
        const float t = 2.0f * u;
        x = t - 1.0f;
      } else {
        x = u;
      }
      X[(lo + v) * ld + c] = x;
    }
  }
}

template <bool MAXCUT>
__global__ __launch_bounds__(256) void k_init_degree(float *__restrict__ X, const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ dmax_p, int64_t lo, int64_t n,
                                                     int32_t ncols, int32_t ld, uint64_t seed, uint64_t traj0,
                                                     float sigma, uint64_t start) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int32_t c = (int32_t)(idx % ncols);
  const int64_t v = idx / ncols;
  const int32_t dmax = *dmax_p;
  const float d = (float)(row_ptr[lo + v + 1] - row_ptr[lo + v]);
  float base = dmax == 0 ? 1.0f : 1.0f - d / (float)dmax;
  if (MAXCUT) base = 2.0f * base - 1.0f;
  uint64_t w[4] = {(uint64_t)v >> 2, traj0 + c, start, 0};
  philox4x64_10(w, seed, PURPOSE_NOISE);
  const uint64_t word = w[v & 3];
  const float u1 = ((float)((uint32_t)word >> 8) + 1.0f) * (1.0f / 16777216.0f);
  const float u2 = (float)((uint32_t)(word >> 32) >> 8) * (1.0f / 16777216.0f);
  const float z = sqrtf(-2.0f * logf(u1)) * cosf(6.283185307179586f * u2);
  X[(lo + v) * ld + c] = clip_box<MAXCUT>(base + sigma * z);
}

__global__ void k_degree_max(const int32_t *__restrict__ row_ptr, int64_t lo, int64_t n, int32_t *out) {
  int32_t m = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    m = max(m, row_ptr[lo + v + 1] - row_ptr[lo + v]);
  atomicMax(out, m);
}

// ---------------------------------------------------------------------------
// fused PGA step: S = A X (CSR order), g, momentum, Pi.  X and Xn differ.
// ---------------------------------------------------------------------------
template <int VEC>
struct VecT;
template <>
struct VecT<1> {
  using T = float;
};
template <>
struct VecT<2> {
  using T = float2;
};
template <>
struct VecT<4> {
  using T = float4;
};

template <int VEC>
__device__ __forceinline__ void load_vec(const float *p, float (&o)[VEC]) {
  if constexpr (VEC == 1) {
    o[0] = *p;
  } else if constexpr (VEC == 2) {
    const float2 t = *reinterpret_cast<const float2 *>(p);
    o[0] = t.x;
    o[1] = t.y;
  } else {
    const float4 t = *reinterpret_cast<const float4 *>(p);
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
  }
}

template <int VEC>
__device__ __forceinline__ void store_vec(float *p, const float (&o)[VEC]) {
  if constexpr (VEC == 1) {
    *p = o[0];
  } else if constexpr (VEC == 2) {
    *reinterpret_cast<float2 *>(p) = make_float2(o[0], o[1]);
  } else {
    *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
  }
}

// acc[i] = sum over the row's neighbours, ascending CSR order, one rounding per add.
// Column indices (and weights) are streamed with non-temporal loads so that
// they do not evict iterate lines.  With 4 or more lanes per row the lanes
// load up to `lanes` indices of the row in one coalesced load and pass them
// round with wave shuffles; then every lane of the row's group must call it
// (lanes whose columns are past the batch pass colok = false and only help
// with the index loads).  With 1 or 2 lanes per row each lane loads eight
// indices at a time and issues the eight gathers back to back.
template <int VEC, bool WEIGHTED>
__device__ __forceinline__ void add_neighbour(float (&acc)[VEC], const float (&x)[VEC], int32_t w) {
  if (WEIGHTED) {
    const float wf = (float)w;
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      const float p = wf * x[i];
      acc[i] = acc[i] + p;
    }
  } else {
#pragma unroll
    for (int i = 0; i < VEC; ++i) acc[i] = acc[i] + x[i];
  }
}

// wsum: the row's weight sum W_v (its degree when unweighted), an exact
// integer sum of the weights the gather loads anyway (valid where colok).
template <int VEC, bool WEIGHTED, int KB = 4>
__device__ __forceinline__ void row_gather(const GraphView &g, const float *__restrict__ X, int64_t v, int32_t col,
                                           int32_t ld, int32_t lanes_log2, bool colok, float (&acc)[VEC],
                                           int32_t &wsum) {
#pragma unroll
  for (int i = 0; i < VEC; ++i) acc[i] = 0.0f;
  const int32_t beg = g.row_ptr[v], end = g.row_ptr[v + 1];
  wsum = WEIGHTED ? 0 : end - beg;
  if (lanes_log2 >= 2) {
    const int32_t lanes = 1 << lanes_log2;
    const int32_t lane = threadIdx.x & (lanes - 1);
    // batches of KB indices: shuffled out first, then KB gathers issued back
    // to back, then added in order (the shuffles keep a plain loop from
    // being unrolled, which would leave one gather in flight per lane);
    // 8 in flight suit rows of very uneven degree (graphs with hubs), 4
    // near-regular ones
    for (int32_t j0 = beg; j0 < end; j0 += lanes) {
      const bool have = j0 + lane < end;
      const int32_t myu = have ? __builtin_nontemporal_load(g.col_idx + j0 + lane) : 0;
      const int32_t myw = WEIGHTED && have ? __builtin_nontemporal_load(g.weight + j0 + lane) : 1;
      const int32_t cnt = min(lanes, end - j0);
      for (int32_t k0 = 0; k0 < cnt; k0 += KB) {
        int64_t u[KB];
        int32_t w[KB];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          const int32_t src = min(k0 + kk, lanes - 1);
          u[kk] = __shfl(myu, src, lanes);
          w[kk] = WEIGHTED ? __shfl(myw, src, lanes) : 1;
        }
        float x[KB][VEC];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
          if (colok && k0 + kk < cnt) load_vec<VEC>(X + u[kk] * ld + col, x[kk]);
#pragma unroll
        for (int kk = 0; kk < KB; ++kk)
          if (colok && k0 + kk < cnt) add_neighbour<VEC, WEIGHTED>(acc, x[kk], w[kk]);
        if (WEIGHTED) {
#pragma unroll
          for (int kk = 0; kk < KB; ++kk)
            if (k0 + kk < cnt) wsum += w[kk];
        }
      }
    }
    return;
  }
  if (!colok) return;
  for (int32_t j0 = beg; j0 < end; j0 += 8) {
    int32_t u[8], w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool ok = j0 + k < end;
      u[k] = ok ? __builtin_nontemporal_load(g.col_idx + j0 + k) : 0;
      w[k] = WEIGHTED && ok ? __builtin_nontemporal_load(g.weight + j0 + k) : 1;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (j0 + k >= end) break;
      float x[VEC];
      load_vec<VEC>(X + (int64_t)u[k] * ld + col, x);
      add_neighbour<VEC, WEIGHTED>(acc, x, w[k]);
      if (WEIGHTED) wsum += w[k];
    }
  }
}

// Two rows of equal degree summed in lockstep by one lane group (4 or more
// lanes per row): twice the independent gathers in flight per lane.  Each
// row's sum keeps its own ascending CSR order.
template <int VEC, bool WEIGHTED>
__device__ __forceinline__ void row_gather2(const GraphView &g, const float *__restrict__ X, int64_t v0, int64_t v1,
                                            int32_t col, int32_t ld, int32_t lanes_log2, bool colok,
                                            float (&a0)[VEC], float (&a1)[VEC], int32_t &ws0, int32_t &ws1) {
#pragma unroll
  for (int i = 0; i < VEC; ++i) {
    a0[i] = 0.0f;
    a1[i] = 0.0f;
  }
  const int32_t b0 = g.row_ptr[v0], e0 = g.row_ptr[v0 + 1];
  const int32_t b1 = g.row_ptr[v1];
  ws0 = WEIGHTED ? 0 : e0 - b0;
  ws1 = ws0;
  const int32_t lanes = 1 << lanes_log2;
  const int32_t lane = threadIdx.x & (lanes - 1);
  for (int32_t j = 0; j < e0 - b0; j += lanes) {
    const int32_t cnt = min(lanes, e0 - b0 - j);
    const bool have = lane < cnt;
    const int32_t u0l = have ? __builtin_nontemporal_load(g.col_idx + b0 + j + lane) : 0;
    const int32_t u1l = have ? __builtin_nontemporal_load(g.col_idx + b1 + j + lane) : 0;
    const int32_t w0l = WEIGHTED && have ? __builtin_nontemporal_load(g.weight + b0 + j + lane) : 1;
    const int32_t w1l = WEIGHTED && have ? __builtin_nontemporal_load(g.weight + b1 + j + lane) : 1;
#pragma unroll 4
    for (int32_t k = 0; k < cnt; ++k) {
      const int64_t u0 = __shfl(u0l, k, lanes), u1 = __shfl(u1l, k, lanes);
      const int32_t w0 = WEIGHTED ? __shfl(w0l, k, lanes) : 1, w1 = WEIGHTED ? __shfl(w1l, k, lanes) : 1;
      if (WEIGHTED) {
        ws0 += w0;
        ws1 += w1;
      }
      if (!colok) continue;
      float x0[VEC], x1[VEC];
      load_vec<VEC>(X + u0 * ld + col, x0);
      load_vec<VEC>(X + u1 * ld + col, x1);
      add_neighbour<VEC, WEIGHTED>(a0, x0, w0);
      add_neighbour<VEC, WEIGHTED>(a1, x1, w1);
    }
  }
}

// ---------------------------------------------------------------------------
// Hub rows.  A row of degree above g.hub_deg (listed in g.hubs) is not
// handled by a lane group: the first hub_blocks(g, ncols) workgroups of a
// launch each take one (hub, slice of HUB_SW columns).  The whole workgroup
// stages the slice of up to HUB_CHUNK neighbours at a time into LDS, then
// lane c of the first wavefront adds column c0 + c in ascending CSR order,
// so the result is the same as row_gather's.
// ---------------------------------------------------------------------------
constexpr int HUB_SW = 4;
constexpr int HUB_CHUNK = 1024;
// dynamic LDS of a hub workgroup
static inline size_t hub_lds(bool weighted) { return HUB_CHUNK * (16 + (weighted ? 4 : 0)); }

__host__ __device__ inline int32_t hub_slices(int32_t ncols) { return (ncols + HUB_SW - 1) / HUB_SW; }
__host__ __device__ inline int64_t hub_blocks(const GraphView &g, int32_t ncols) {
  return (int64_t)g.nhub * hub_slices(ncols);
}

struct HubItem {
  int64_t v;   // global row
  int32_t h;   // index in the graph's hub list
  int32_t c0;  // first column of the slice
  int32_t cw;  // columns in the slice
};

__device__ __forceinline__ HubItem hub_item(const GraphView &g, int32_t ncols, int64_t bx) {
  HubItem it;
  const int32_t ns = hub_slices(ncols);
  it.h = (int32_t)(bx / ns);
  it.c0 = (int32_t)(bx % ns) * HUB_SW;
  it.cw = min(HUB_SW, ncols - it.c0);
  it.v = g.hubs[it.h];
  return it;
}

// Every thread of the workgroup calls it; the sum is valid in threads 0 .. cw-1.
template <bool WEIGHTED>
__device__ __forceinline__ float hub_gather(const GraphView &g, const float *__restrict__ X, const HubItem &it,
                                            int32_t ld) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  float4 *st = reinterpret_cast<float4 *>(dyn_lds);          // [HUB_CHUNK]
  float *wst = reinterpret_cast<float *>(st + HUB_CHUNK);  // [HUB_CHUNK] when weighted
  const int32_t beg = g.row_ptr[it.v], end = g.row_ptr[it.v + 1];
  const bool v4 = it.cw == 4 && (ld & 3) == 0 && ((uintptr_t)X & 15) == 0;
  const float *sf = reinterpret_cast<const float *>(st);
  float acc = 0.0f;
  for (int32_t j0 = beg; j0 < end; j0 += HUB_CHUNK) {
    const int32_t cnt = min(HUB_CHUNK, end - j0);
    for (int32_t k = threadIdx.x; k < cnt; k += blockDim.x) {
      const int64_t u = __builtin_nontemporal_load(g.col_idx + j0 + k);
      const float *p = X + u * ld + it.c0;
      float4 x;
      if (v4) {
        x = *reinterpret_cast<const float4 *>(p);
      } else {
        x.x = p[0];
        x.y = it.cw > 1 ? p[1] : 0.0f;
        x.z = it.cw > 2 ? p[2] : 0.0f;
        x.w = it.cw > 3 ? p[3] : 0.0f;
      }
      st[k] = x;
      if (WEIGHTED) wst[k] = (float)g.weight[j0 + k];
    }
    __syncthreads();
    if ((int32_t)threadIdx.x < it.cw) {
#pragma unroll 8
      for (int32_t k = 0; k < cnt; ++k) {
        const float x = sf[k * 4 + threadIdx.x];
        if (WEIGHTED) {
          const float p = wst[k] * x;
          acc = acc + p;
        } else {
          acc = acc + x;
        }
      }
    }
    __syncthreads();
  }
  return acc;
}

// The rows a lane group skips because a hub workgroup owns them.
__device__ __forceinline__ bool is_hub_row(const GraphView &g, int64_t v) {
  return g.nhub > 0 && g.row_ptr[v + 1] - g.row_ptr[v] > g.hub_deg;
}

// The ROWS rows of a lane group in row workgroup bx (rows grp and grp + rpb
// of a ROWS * rpb-row block; rpb = lane groups per workgroup), whether the
// group owns each (in range, not a hub; uniform over the group), their
// neighbour sums and their weight sums W_v.  Every lane of the group must call it.  ROWS = 2 is
// launched for near-regular graphs only: two rows of equal degree go in
// lockstep, otherwise one after the other.
template <int VEC, bool WEIGHTED, int ROWS, int KB = 4>
__device__ __forceinline__ void group_gather(const GraphView &g, const float *__restrict__ X, int64_t bx, int32_t by,
                                             int32_t ncols, int32_t ld, int32_t lanes_log2, int64_t (&v)[ROWS],
                                             bool (&own)[ROWS], int32_t &col, float (&acc)[ROWS][VEC],
                                             int32_t (&wsum)[ROWS]) {
  const int32_t lanes = 1 << lanes_log2;
  const int32_t rpb = blockDim.x >> lanes_log2;
  const int64_t r0 = bx * ROWS * rpb + (threadIdx.x >> lanes_log2);
  col = (int32_t)(by * lanes + (threadIdx.x & (lanes - 1))) * VEC;
  const bool colok = col < ncols;
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    const int64_t r = r0 + (int64_t)k * rpb;
    v[k] = g.lo + r;
    own[k] = r < g.n && !is_hub_row(g, v[k]);
    wsum[k] = 0;
  }
  if constexpr (ROWS == 2) {
    if (own[0] && own[1] &&
        g.row_ptr[v[0] + 1] - g.row_ptr[v[0]] == g.row_ptr[v[1] + 1] - g.row_ptr[v[1]]) {
      row_gather2<VEC, WEIGHTED>(g, X, v[0], v[1], col, ld, lanes_log2, colok, acc[0], acc[1], wsum[0], wsum[1]);
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < ROWS; ++k)
    if (own[k]) row_gather<VEC, WEIGHTED, KB>(g, X, v[k], col, ld, lanes_log2, colok, acc[k], wsum[k]);
}

// W_v, the row's weight sum (its degree when unweighted), for f_L and f_P
// on hub rows (lane groups take it from their gather)
template <bool WEIGHTED>
__device__ __forceinline__ float weighted_degree(const GraphView &g, int64_t v) {
  const int32_t beg = g.row_ptr[v], end = g.row_ptr[v + 1];
  if (!WEIGHTED) return (float)(end - beg);
  int32_t w = 0;
  for (int32_t j = beg; j < end; ++j) w += g.weight[j];
  return (float)w;
}

// One PGA step of Sec. 3 (with optional heavy-ball momentum) for a single column.
template <int OBJ, bool MOMENTUM>
__device__ __forceinline__ void step_update(float &x, float &vv, float acc, float W, float alpha, float mu,
                                            float param) {
  constexpr bool MAXCUT = OBJ != OBJ_H;
  const float gr = grad_of<OBJ>(acc, x, W, param);
  float d = gr;
  if (MOMENTUM) {
    const float t = mu * vv;
    vv = t + gr;
    d = vv;
  }
  const float s = alpha * d;
  const float y = x + s;
  x = clip_box<MAXCUT>(y);
}

// colact[c] = 0 marks a trajectory that stopped stepping for the rest of
// the round (early exit): its iterate and momentum are copied through.
// nullptr = all active.
template <int VEC, int OBJ, bool WEIGHTED, bool MOMENTUM, int ROWS, int KB = 4>
__global__ __launch_bounds__(256) void k_pga_step(GraphView g, const float *__restrict__ X, float *__restrict__ Xn,
                                                  float *__restrict__ V, int32_t ncols, int32_t ld,
                                                  int32_t lanes_log2, float alpha, float mu, float param,
                                                  const int8_t *__restrict__ colact) {
  const int64_t nhb = hub_blocks(g, ncols);
  const Blk blk = xcd_blk(g.xcd_local);
  if (blk.x < nhb) {
    if (blk.y != 0) return;
    const HubItem it = hub_item(g, ncols, blk.x);
    const float acc = hub_gather<WEIGHTED>(g, X, it, ld);
    if ((int32_t)threadIdx.x < it.cw) {
      const int64_t e = it.v * ld + it.c0 + threadIdx.x;
      float x = X[e], vv = MOMENTUM ? V[e] : 0.0f;
      const float W = OBJ == OBJ_FL || OBJ == OBJ_FP ? weighted_degree<WEIGHTED>(g, it.v) : 0.0f;
      if (!colact || colact[it.c0 + threadIdx.x]) step_update<OBJ, MOMENTUM>(x, vv, acc, W, alpha, mu, param);
      Xn[e] = x;
      if (MOMENTUM) V[e] = vv;
    }
    return;
  }
  int64_t v[ROWS];
  bool own[ROWS];
  int32_t col;
  float acc[ROWS][VEC];
  int32_t wsum[ROWS];
  group_gather<VEC, WEIGHTED, ROWS, KB>(g, X, blk.x - nhb, blk.y, ncols, ld, lanes_log2, v, own, col, acc, wsum);
  if (col >= ncols) return;
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    if (!own[k]) continue;
    float x[VEC], vv[VEC];
    load_vec<VEC>(X + v[k] * ld + col, x);
    if (MOMENTUM) load_vec<VEC>(V + v[k] * ld + col, vv);
    const float W = OBJ == OBJ_FL || OBJ == OBJ_FP ? (float)wsum[k] : 0.0f;
#pragma unroll
    for (int i = 0; i < VEC; ++i)
      if (!colact || colact[col + i]) step_update<OBJ, MOMENTUM>(x[i], vv[i], acc[k][i], W, alpha, mu, param);
    store_vec<VEC>(Xn + v[k] * ld + col, x);
    if (MOMENTUM) store_vec<VEC>(V + v[k] * ld + col, vv);
  }
}

__global__ void k_copy_f32(const float *__restrict__ a, float *__restrict__ b, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_strided_copy_f32(const float *__restrict__ src, int32_t lds, int32_t cs, float *__restrict__ dst,
                                   int32_t ldd, int32_t cd, int64_t lo, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) dst[(lo + v) * ldd + cd] = src[(lo + v) * lds + cs];
}

__global__ void k_strided_copy_i8(const int8_t *__restrict__ src, int32_t lds, int32_t cs, int8_t *__restrict__ dst,
                                  int32_t ldd, int32_t cd, int64_t lo, int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) dst[(lo + v) * ldd + cd] = src[(lo + v) * lds + cs];
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_fill_i64(int64_t *p, int64_t count, int64_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_fill_f32(float *p, int64_t count, float value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---------------------------------------------------------------------------
// rounding and exact evaluation
// ---------------------------------------------------------------------------
template <bool MAXCUT>
__global__ __launch_bounds__(256) void k_round(const float *__restrict__ X, int8_t *__restrict__ Z, int64_t lo,
                                               int64_t n, int32_t ncols, int32_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t v = lo + idx / ncols;
  const int32_t c = (int32_t)(idx % ncols);
  Z[v * ld + c] = round_x<MAXCUT>(X[v * ld + c]);
}

// VEC int8 states from p (4-byte aligned when VEC = 4), sign-extended
template <int VEC>
__device__ __forceinline__ void load_z(const int8_t *p, int32_t (&z)[VEC]) {
  if constexpr (VEC == 4) {
    const uint32_t w = *reinterpret_cast<const uint32_t *>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) z[i] = (int32_t)(int8_t)(w >> (8 * i));
  } else {
#pragma unroll
    for (int i = 0; i < VEC; ++i) z[i] = p[i];
  }
}

// NB = A Z (int32) and per-column accumulators acc[3][ncols] (int64):
// MIS  : acc0 = |I|, acc1 = sum z m = 2 * edges inside I, acc2 = #{v: z=0, m=0}
// MaxCut: acc0 = sum_v (W_v - s_v t_v) = 4 Cut(S)   (W_v = sum of row weights),
//         acc1 = #{v: the projected step would move s_v}
// Each lane takes VEC consecutive columns (VEC = 4: one 4-byte state load
// per neighbour, one 16-byte count store; needs ncols, ld multiples of 4).
template <bool MAXCUT, bool WEIGHTED, int VEC>
__global__ __launch_bounds__(256) void k_nbr_eval(GraphView g, const int8_t *__restrict__ Z, int32_t *__restrict__ NB,
                                                  unsigned long long *__restrict__ acc, int32_t ncols, int32_t ld,
                                                  int32_t lanes_log2) {
  // per-column sums: wavefront shuffle reduction over the lanes of one column,
  // then one LDS add per (wavefront, column) and one global atomic per
  // (block, column)
  constexpr int SC = 64 * VEC;  // columns of a workgroup's slice, at most
  __shared__ long long sacc[3][SC];
  const int lanes = 1 << lanes_log2;
  for (int t = threadIdx.x; t < 3 * SC; t += blockDim.x) sacc[t / SC][t % SC] = 0;
  __syncthreads();
  // grid-stride over the row workgroups, so that the per-column global
  // atomics are paid once per resident workgroup, not once per 256 rows
  const int64_t nrb = (g.n + (blockDim.x >> lanes_log2) - 1) / (blockDim.x >> lanes_log2);
  long long a[3][VEC];
#pragma unroll
  for (int i = 0; i < VEC; ++i) a[0][i] = a[1][i] = a[2][i] = 0;
  for (int64_t bx = blockIdx.x; bx < nrb; bx += gridDim.x) {
    const RowMap m = map_rows<VEC>(g.n, ncols, lanes_log2, bx);
    if (!m.active) continue;
    const int64_t v = g.lo + m.row;
    const int32_t beg = g.row_ptr[v], end = g.row_ptr[v + 1];
    int32_t s[VEC], wsum = 0;
#pragma unroll
    for (int i = 0; i < VEC; ++i) s[i] = 0;
#pragma unroll 4
    for (int32_t j = beg; j < end; ++j) {
      const int64_t u = __builtin_nontemporal_load(g.col_idx + j);
      int32_t zu[VEC];
      load_z<VEC>(Z + u * ld + m.col, zu);
      if (WEIGHTED) {
        const int32_t w = __builtin_nontemporal_load(g.weight + j);
#pragma unroll
        for (int i = 0; i < VEC; ++i) s[i] += w * zu[i];
        wsum += w;
      } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) s[i] += zu[i];
      }
    }
    if (!WEIGHTED) wsum = end - beg;
    if (NB) {
      if constexpr (VEC == 4)
        *reinterpret_cast<int4 *>(NB + v * ld + m.col) = make_int4(s[0], s[1], s[2], s[3]);
      else
#pragma unroll
        for (int i = 0; i < VEC; ++i) NB[v * ld + m.col + i] = s[i];
    }
    int32_t zv[VEC];
    load_z<VEC>(Z + v * ld + m.col, zv);
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      if (MAXCUT) {
        a[0][i] += (long long)wsum - (long long)zv[i] * s[i];
        // the projected f_B step moves s_v off the vertex unless s_v t_v < 0,
        // or s_v t_v = 0 and s_v = -1 (gradient -lambda - 2 t_v, 0 < lambda < 2)
        const int32_t st = zv[i] * s[i];
        a[1][i] += (st > 0 || (st == 0 && zv[i] == 1)) ? 1 : 0;
      } else {
        a[0][i] += zv[i];
        a[1][i] += zv[i] ? s[i] : 0;
        a[2][i] += (zv[i] == 0 && s[i] == 0) ? 1 : 0;
      }
    }
  }
  const int width = lanes < 64 ? lanes : 64;
  const int wl = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < (MAXCUT ? 2 : 3); ++k)
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      const long long t = wave_sum_stride(a[k][i], width);
      if (wl < width && t)
        atomicAdd(reinterpret_cast<unsigned long long *>(&sacc[k][wl * VEC + i]), (unsigned long long)t);
    }
  __syncthreads();
  for (int t = threadIdx.x; t < lanes * VEC; t += blockDim.x) {
    const int32_t c = blockIdx.y * lanes * VEC + t;
    if (c < ncols) {
      for (int k = 0; k < (MAXCUT ? 2 : 3); ++k)
        if (sacc[k][t]) atomicAdd(&acc[k * ncols + c], (unsigned long long)sacc[k][t]);
    }
  }
}

template <bool MAXCUT>
__global__ void k_value_finalize(const long long *__restrict__ acc, int32_t ncols, int64_t *__restrict__ value,
                                 int64_t *__restrict__ conflicts, int8_t *__restrict__ fixed) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  if (MAXCUT) {
    value[c] = acc[c] / 4;
    if (fixed) fixed[c] = acc[ncols + c] == 0 ? 1 : 0;
  } else {
    const long long size = acc[c], conf = acc[ncols + c] / 2, freev = acc[2 * ncols + c];
    value[c] = conf == 0 ? size : -1;
    if (conflicts) conflicts[c] = conf;
    if (fixed) fixed[c] = (conf == 0 && freev == 0) ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// 1-flip local search, parallel rule
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ls_prio(uint32_t *__restrict__ PRIO, int64_t lo, int64_t n, int32_t ncols,
                                                 int32_t ld, uint64_t seed, uint64_t traj0, uint64_t round,
                                                 uint64_t purpose) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nvb = (n + 7) >> 3;
  if (idx >= nvb * ncols) return;
  const int32_t c = (int32_t)(idx % ncols);
  const int64_t vb = idx / ncols;
  uint32_t r[8];
  philox_block8(r, seed, purpose, traj0 + c, round, (uint64_t)vb);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t v = vb * 8 + i;
    if (v < n) PRIO[(lo + v) * ld + c] = r[i];
  }
}

// F[v] = v in P and its key beats every neighbour in P.  active[0] is set
// when P is non-empty.  When prev_active is given and *prev_active == 0
// the search has already stopped and the kernel does nothing.
template <bool MAXCUT>
__global__ __launch_bounds__(256) void k_ls_select(GraphView g, const int8_t *__restrict__ Z,
                                                   const int32_t *__restrict__ NB, const uint32_t *__restrict__ PRIO,
                                                   int8_t *__restrict__ F, int32_t *active,
                                                   const int32_t *prev_active, int32_t ncols, int32_t ld,
                                                   int32_t lanes_log2) {
  if (prev_active && *prev_active == 0) return;
  const RowMap m = map_rows<1>(g.n, ncols, lanes_log2);
  if (!m.active) return;
  const int64_t v = g.lo + m.row;
  const int64_t e = v * ld + m.col;
  int32_t k1;
  const bool p = ls_candidate_t<MAXCUT>(Z[e], NB[e], k1);
  int8_t f = 0;
  // one store of the "still searching" flag per wavefront
  const unsigned long long bal = __ballot(p);
  if (p && (int)(threadIdx.x & 63) == __builtin_ctzll(bal)) *active = 1;
  if (p) {
    const uint32_t pv = PRIO[e];
    f = 1;
    const int32_t beg = g.row_ptr[v], end = g.row_ptr[v + 1];
    for (int32_t j = beg; j < end; ++j) {
      const int64_t u = g.col_idx[j];
      const int64_t eu = u * ld + m.col;
      int32_t k1u;
      if (ls_candidate_t<MAXCUT>(Z[eu], NB[eu], k1u) && key_beats(k1u, PRIO[eu], u, k1, pv, v)) {
        f = 0;
        break;
      }
    }
  }
  F[e] = f;
}

template <bool MAXCUT, bool WEIGHTED>
__global__ __launch_bounds__(256) void k_ls_apply(GraphView g, const int8_t *__restrict__ F, int8_t *__restrict__ Z,
                                                  int32_t *__restrict__ NB, const int32_t *active, int32_t ncols,
                                                  int32_t ld, int32_t lanes_log2) {
  if (*active == 0) return;
  const RowMap m = map_rows<1>(g.n, ncols, lanes_log2);
  if (!m.active) return;
  const int64_t v = g.lo + m.row;
  const int64_t e = v * ld + m.col;
  if (!F[e]) return;
  const int32_t z = Z[e];
  const int32_t zn = MAXCUT ? -z : 1 - z;
  Z[e] = (int8_t)zn;
  const int32_t d = zn - z;
  const int32_t beg = g.row_ptr[v], end = g.row_ptr[v + 1];
  for (int32_t j = beg; j < end; ++j) {
    const int64_t u = g.col_idx[j];
    atomicAdd(&NB[u * ld + m.col], WEIGHTED ? d * g.weight[j] : d);
  }
}

// The same iteration with one wavefront per (row v, 64 columns), for graphs
// of large mean degree.  When few of the 64 columns move (the usual case
// once the search has settled) each candidate column's neighbours are tested
// 64 at a time, one lane per neighbour and a ballot, and a flipped column's
// count updates are issued 64 at a time; with many, every lane walks the
// row for its own column as above.  F and the updates are the same either
// way: a candidate wins iff no neighbouring candidate has a larger key.
constexpr int LS_ROW_FEW = 16;

template <bool MAXCUT>
__global__ __launch_bounds__(256) void k_ls_select_rows(GraphView g, const int8_t *__restrict__ Z,
                                                        const int32_t *__restrict__ NB,
                                                        const uint32_t *__restrict__ PRIO, int8_t *__restrict__ F,
                                                        int32_t *active, const int32_t *prev_active, int32_t ncols,
                                                        int32_t ld) {
  if (prev_active && *prev_active == 0) return;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= g.n) return;  // the whole wavefront
  const int32_t lane = threadIdx.x & 63;
  const int32_t c0 = (int32_t)blockIdx.y * 64;
  const int32_t cc = ncols - c0 < 64 ? ncols - c0 : 64;
  const int32_t v = __builtin_amdgcn_readfirstlane((int32_t)(g.lo + row));
  const int64_t e = (int64_t)v * ld + c0 + lane;
  int32_t k1 = 0;
  const bool p = lane < cc && ls_candidate_t<MAXCUT>(Z[e], NB[e], k1);
  const uint32_t pv = p ? PRIO[e] : 0u;
  unsigned long long cand = __ballot(p);
  if (p && lane == __builtin_ctzll(cand)) *active = 1;
  bool win = p;
  if (cand) {
    const int32_t vb = __builtin_amdgcn_readfirstlane(g.row_ptr[v]);
    const int32_t vd = __builtin_amdgcn_readfirstlane(g.row_ptr[v + 1]) - vb;
    if (__builtin_popcountll(cand) > LS_ROW_FEW) {
      if (p) {
        const int64_t col = c0 + lane;
        for (int32_t j = 0; j < vd; ++j) {
          const int32_t u = g.col_idx[vb + j];
          const int64_t eu = (int64_t)u * ld + col;
          int32_t k1u;
          if (ls_candidate_t<MAXCUT>(Z[eu], NB[eu], k1u) && key_beats(k1u, PRIO[eu], u, k1, pv, v)) {
            win = false;
            break;
          }
        }
      }
    } else {
      // the row's first 128 neighbours stay in registers across columns
      const int32_t u0 = lane < vd ? g.col_idx[vb + lane] : 0;
      const int32_t u1 = 64 + lane < vd ? g.col_idx[vb + 64 + lane] : 0;
      while (cand) {
        const int32_t c = __builtin_ctzll(cand);
        cand &= cand - 1;
        const int64_t col = c0 + c;
        const int32_t k1c = __builtin_amdgcn_readlane(k1, c);
        const uint32_t pvc = (uint32_t)__builtin_amdgcn_readlane((int32_t)pv, c);
        bool lose = false;
        for (int32_t m = 0; m < vd && !lose; m += 64) {
          bool beats = false;
          if (m + lane < vd) {
            const int32_t u = m == 0 ? u0 : m == 64 ? u1 : g.col_idx[vb + m + lane];
            const int64_t eu = (int64_t)u * ld + col;
            int32_t k1u;
            beats = ls_candidate_t<MAXCUT>(Z[eu], NB[eu], k1u) && key_beats(k1u, PRIO[eu], u, k1c, pvc, v);
          }
          lose = __ballot(beats) != 0;
        }
        if (lane == c) win = !lose;
      }
    }
  }
  if (lane < cc) F[e] = win ? 1 : 0;
}

template <bool MAXCUT, bool WEIGHTED>
__global__ __launch_bounds__(256) void k_ls_apply_rows(GraphView g, const int8_t *__restrict__ F,
                                                       int8_t *__restrict__ Z, int32_t *__restrict__ NB,
                                                       const int32_t *active, int32_t ncols, int32_t ld) {
  if (*active == 0) return;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= g.n) return;  // the whole wavefront
  const int32_t lane = threadIdx.x & 63;
  const int32_t c0 = (int32_t)blockIdx.y * 64;
  const int32_t cc = ncols - c0 < 64 ? ncols - c0 : 64;
  const int32_t v = __builtin_amdgcn_readfirstlane((int32_t)(g.lo + row));
  const int64_t e = (int64_t)v * ld + c0 + lane;
  const bool f = lane < cc && F[e] != 0;
  int32_t d = 0;
  if (f) {
    const int32_t z = Z[e];
    const int32_t zn = MAXCUT ? -z : 1 - z;
    Z[e] = (int8_t)zn;
    d = zn - z;
  }
  unsigned long long fl = __ballot(f);
  if (!fl) return;
  const int32_t vb = __builtin_amdgcn_readfirstlane(g.row_ptr[v]);
  const int32_t vd = __builtin_amdgcn_readfirstlane(g.row_ptr[v + 1]) - vb;
  if (__builtin_popcountll(fl) > LS_ROW_FEW) {
    if (f)
      for (int32_t j = 0; j < vd; ++j)
        atomicAdd(&NB[(int64_t)g.col_idx[vb + j] * ld + c0 + lane], WEIGHTED ? d * g.weight[vb + j] : d);
    return;
  }
  while (fl) {
    const int32_t c = __builtin_ctzll(fl);
    fl &= fl - 1;
    const int32_t dc = __builtin_amdgcn_readlane(d, c);
    for (int32_t m = lane; m < vd; m += 64)
      atomicAdd(&NB[(int64_t)g.col_idx[vb + m] * ld + c0 + c], WEIGHTED ? dc * g.weight[vb + m] : dc);
  }
}

// ---------------------------------------------------------------------------
// pair moves of the paper's own searches, parallel rule: the (1,2)-swap of
// Def. 2.3 (MIS) and the 2-flip of Def. 2.5 (MaxCut).  One thread per
// (vertex, column); every array is [n][ld], one column per trajectory.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool has_edge(const GraphView &g, int32_t a, int32_t b) {
  // rows are strictly ascending
  int32_t lo = g.row_ptr[a], hi = g.row_ptr[a + 1];
  const int32_t end = hi;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (g.col_idx[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo < end && g.col_idx[lo] == b;
}

__global__ __launch_bounds__(256) void k_fill_rows_i32(int32_t *__restrict__ A, int64_t lo, int64_t n, int32_t v,
                                                       int32_t ncols, int32_t ld, int32_t lanes_log2) {
  const RowMap m = map_rows<1>(n, ncols, lanes_log2);
  if (m.active) A[(lo + m.row) * ld + m.col] = v;
}

// Tightness bits: word (u, chunk) bit l = 1 iff column 64 chunk + l has
// z_u = 0 and m_u = 1 (u is outside I with exactly one neighbour in I).
// One wavefront per (row, chunk of 64 columns).
__global__ __launch_bounds__(256) void k_tight_bits(GraphView g, const int8_t *__restrict__ Z,
                                                    const int32_t *__restrict__ NB,
                                                    unsigned long long *__restrict__ TB, int32_t ncols, int32_t ld) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= g.n) return;  // the whole wavefront
  const int32_t lane = threadIdx.x & 63;
  const int32_t col = (int32_t)blockIdx.y * 64 + lane;
  bool t = false;
  if (col < ncols) {
    const int64_t e = (g.lo + row) * ld + col;
    t = Z[e] == 0 && NB[e] == 1;
  }
  const unsigned long long bal = __ballot(t);
  if (lane == 0) TB[(g.lo + row) * gridDim.y + blockIdx.y] = bal;
}

// v in I proposes the first pair (u, w) of its neighbours in CSR order with
// m_u = m_w = 1 (v is their only neighbour in I) and u, w not adjacent:
// then I - v + u + w is independent.  PU/PW = u, w or -1; OWN[u] = OWN[w] = v.
// One wavefront per (row v, chunk of 64 columns); its lanes span v's
// neighbour positions, 64 at a time.  For each column with v in I the
// tight positions come from one ballot per neighbour chunk over the
// tightness words (k_tight_bits, 64 columns per chunk), and the partners of
// a tight u are tested for adjacency in parallel, the lowest position
// winning; so the first pair in CSR order is found in a few wavefront-wide
// steps.
__global__ __launch_bounds__(256) void k_swap_propose(GraphView g, const int8_t *__restrict__ Z,
                                                      const unsigned long long *__restrict__ TB,
                                                      int32_t *__restrict__ PU, int32_t *__restrict__ PW,
                                                      int32_t *__restrict__ OWN, int32_t ncols, int32_t ld) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= g.n) return;  // the whole wavefront
  const int32_t lane = threadIdx.x & 63;
  const int32_t c0 = (int32_t)blockIdx.y * 64;
  const int32_t cc = ncols - c0 < 64 ? ncols - c0 : 64;  // columns in this chunk
  const int64_t nchunk = gridDim.y;
  const int32_t v = __builtin_amdgcn_readfirstlane((int32_t)(g.lo + row));
  const int64_t e = (int64_t)v * ld + c0 + lane;
  const bool in_i = lane < cc && Z[e] == 1;
  unsigned long long act = __ballot(in_i);
  const int32_t beg = __builtin_amdgcn_readfirstlane(g.row_ptr[v]);
  const int32_t deg = __builtin_amdgcn_readfirstlane(g.row_ptr[v + 1]) - beg;
  const int32_t nk = (deg + 63) >> 6;
  // The row's neighbours and their tightness words do not depend on the
  // column: the first 128 are loaded once per wavefront into registers.
  int32_t ru0 = 0, ru1 = 0;
  unsigned long long rt0 = 0ull, rt1 = 0ull;
  if (act) {  // uniform: some column has v in I
    if (lane < deg) {
      ru0 = g.col_idx[beg + lane];
      rt0 = TB[(int64_t)ru0 * nchunk + blockIdx.y];
    }
    if (nk > 1 && 64 + lane < deg) {
      ru1 = g.col_idx[beg + 64 + lane];
      rt1 = TB[(int64_t)ru1 * nchunk + blockIdx.y];
    }
  }
  // neighbour chunk k of the row: its ids and tightness words (0 past the row)
  auto chunk = [&](int32_t k, int32_t &uk, unsigned long long &tk) {
    if (k == 0) {
      uk = ru0;
      tk = rt0;
    } else if (k == 1) {
      uk = ru1;
      tk = rt1;
    } else {
      const int32_t pk = 64 * k + lane;
      uk = pk < deg ? g.col_idx[beg + pk] : 0;
      tk = pk < deg ? TB[(int64_t)uk * nchunk + blockIdx.y] : 0ull;
    }
  };
  int32_t my_u = -1, my_w = -1;  // lane l: result of column c0 + l
  while (act) {
    const int32_t c = __builtin_ctzll(act);
    act &= act - 1;
    bool found = false;
    int32_t fu = -1, fw = -1;
    for (int32_t k = 0; k < nk && !found; ++k) {
      int32_t uk;
      unsigned long long tbk;
      chunk(k, uk, tbk);
      unsigned long long mk = __ballot(((tbk >> c) & 1ull) != 0);
      while (mk && !found) {
        const int32_t i = __builtin_ctzll(mk);
        mk &= mk - 1;
        const int32_t u = __builtin_amdgcn_readlane(uk, i);
        // u's row across the lanes (the first 128 neighbours kept in
        // registers); a partner w is adjacent to u iff some lane holds w
        const int32_t ub = __builtin_amdgcn_readfirstlane(g.row_ptr[u]);
        const int32_t ud = __builtin_amdgcn_readfirstlane(g.row_ptr[u + 1]) - ub;
        const int32_t un0 = lane < ud ? g.col_idx[ub + lane] : -1;
        const int32_t un1 = 64 + lane < ud ? g.col_idx[ub + 64 + lane] : -1;
        for (int32_t k2 = k; k2 < nk && !found; ++k2) {
          int32_t w2;
          unsigned long long tb2;
          chunk(k2, w2, tb2);
          const bool t2 = (k2 > k || lane > i) && ((tb2 >> c) & 1ull);
          unsigned long long cm = __ballot(t2);  // candidate partners, in CSR order
          while (cm && !found) {
            const int32_t j = __builtin_ctzll(cm);
            cm &= cm - 1;
            const int32_t w = __builtin_amdgcn_readlane(w2, j);
            bool adj = __ballot(un0 == w || un1 == w) != 0;
            for (int32_t m = 128; m < ud && !adj; m += 64) {
              const int32_t x = m + lane < ud ? g.col_idx[ub + m + lane] : -1;
              adj = __ballot(x == w) != 0;
            }
            if (!adj) {
              fu = u;
              fw = w;
              found = true;
            }
          }
        }
      }
    }
    if (lane == c) {
      my_u = fu;
      my_w = fw;
    }
  }
  if (lane >= cc) return;
  if (my_u >= 0) {
    OWN[(int64_t)my_u * ld + c0 + lane] = v;
    OWN[(int64_t)my_w * ld + c0 + lane] = v;
  }
  PU[e] = my_u;
  PW[e] = my_w;
}

// The same proposals with one thread per (v, column), for graphs of small
// degree, where a wavefront per row would leave most lanes idle.
__global__ __launch_bounds__(256) void k_swap_propose_lanes(GraphView g, const int8_t *__restrict__ Z,
                                                            const unsigned long long *__restrict__ TB,
                                                            int32_t *__restrict__ PU, int32_t *__restrict__ PW,
                                                            int32_t *__restrict__ OWN, int32_t ncols, int32_t ld,
                                                            int32_t lanes_log2) {
  const RowMap m = map_rows<1>(g.n, ncols, lanes_log2);
  if (!m.active) return;
  const int64_t v = g.lo + m.row;
  const int64_t e = v * ld + m.col;
  const int64_t nchunk = (ncols + 63) >> 6;
  const int64_t chunk = m.col >> 6;
  const int32_t bit = m.col & 63;
  auto tight = [&](int32_t u) { return ((TB[(int64_t)u * nchunk + chunk] >> bit) & 1ull) != 0; };
  int32_t pu = -1, pw = -1;
  if (Z[e] == 1) {
    const int32_t beg = g.row_ptr[v], end = g.row_ptr[v + 1];
    for (int32_t i = beg; i < end && pu < 0; ++i) {
      const int32_t u = g.col_idx[i];
      if (!tight(u)) continue;
      for (int32_t j = i + 1; j < end; ++j) {
        const int32_t w = g.col_idx[j];
        if (tight(w) && !has_edge(g, u, w)) {
          pu = u;
          pw = w;
          break;
        }
      }
    }
    if (pu >= 0) {
      OWN[(int64_t)pu * ld + m.col] = (int32_t)v;
      OWN[(int64_t)pw * ld + m.col] = (int32_t)v;
    }
  }
  PU[e] = pu;
  PW[e] = pw;
}

// A proposal is applied (F = 1) when its key (prio_v, -v) beats the key of
// every other proposal owning a neighbour of u or w.
__global__ __launch_bounds__(256) void k_swap_select(GraphView g, const int32_t *__restrict__ PU,
                                                     const int32_t *__restrict__ PW, const int32_t *__restrict__ OWN,
                                                     const uint32_t *__restrict__ PRIO, int8_t *__restrict__ F,
                                                     int32_t *active, int32_t ncols, int32_t ld, int32_t lanes_log2) {
  const RowMap m = map_rows<1>(g.n, ncols, lanes_log2);
  if (!m.active) return;
  const int64_t v = g.lo + m.row;
  const int64_t e = v * ld + m.col;
  const int32_t pu = PU[e];
  bool f = pu >= 0;
  if (f) {
    const uint32_t pv = PRIO[e];
    const int32_t pw = PW[e];
    for (int k = 0; k < 2 && f; ++k) {
      const int32_t x = k ? pw : pu;
      const int32_t beg = g.row_ptr[x], end = g.row_ptr[x + 1];
      for (int32_t j = beg; j < end; ++j) {
        const int32_t o = OWN[(int64_t)g.col_idx[j] * ld + m.col];
        if (o >= 0 && o != v && key_beats(0, PRIO[(int64_t)o * ld + m.col], o, 0, pv, v)) {
          f = false;
          break;
        }
      }
    }
  }
  const unsigned long long bal = __ballot(f);
  if (f && (int)(threadIdx.x & 63) == __builtin_ctzll(bal)) *active = 1;
  F[e] = f ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_swap_apply(GraphView g, const int8_t *__restrict__ F,
                                                    const int32_t *__restrict__ PU, const int32_t *__restrict__ PW,
                                                    int8_t *__restrict__ Z, int32_t *__restrict__ NB,
                                                    const int32_t *active, int32_t ncols, int32_t ld,
                                                    int32_t lanes_log2) {
  if (*active == 0) return;
  const RowMap m = map_rows<1>(g.n, ncols, lanes_log2);
  if (!m.active) return;
  const int64_t v = g.lo + m.row;
  const int64_t e = v * ld + m.col;
  if (!F[e]) return;
  const int32_t x3[3] = {(int32_t)v, PU[e], PW[e]};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int32_t x = x3[k];
    const int32_t d = k ? 1 : -1;
    Z[(int64_t)x * ld + m.col] = (int8_t)(k ? 1 : 0);
    const int32_t beg = g.row_ptr[x], end = g.row_ptr[x + 1];
    for (int32_t j = beg; j < end; ++j) atomicAdd(&NB[(int64_t)g.col_idx[j] * ld + m.col], d);
  }
}

// The same selection and application with one wavefront per (row v, 64
// columns), for graphs of large mean degree: each proposing column's
// inserted vertices are scanned with the lanes over their neighbours (one
// coalesced index load and one owner gather per 64 neighbours) instead of
// one lane walking 2 x degree neighbours, and the neighbour-count updates
// of a winner are issued 64 at a time.
__global__ __launch_bounds__(256) void k_swap_select_rows(GraphView g, const int32_t *__restrict__ PU,
                                                          const int32_t *__restrict__ PW,
                                                          const int32_t *__restrict__ OWN,
                                                          const uint32_t *__restrict__ PRIO, int8_t *__restrict__ F,
                                                          int32_t *active, int32_t ncols, int32_t ld) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= g.n) return;  // the whole wavefront
  const int32_t lane = threadIdx.x & 63;
  const int32_t c0 = (int32_t)blockIdx.y * 64;
  const int32_t cc = ncols - c0 < 64 ? ncols - c0 : 64;
  const int32_t v = __builtin_amdgcn_readfirstlane((int32_t)(g.lo + row));
  const int64_t e = (int64_t)v * ld + c0 + lane;
  const int32_t pu = lane < cc ? PU[e] : -1;
  const int32_t pw = lane < cc ? PW[e] : -1;
  const uint32_t pv = lane < cc ? PRIO[e] : 0u;
  bool win = pu >= 0;
  unsigned long long prop = __ballot(pu >= 0);
  while (prop) {
    const int32_t c = __builtin_ctzll(prop);
    prop &= prop - 1;
    const int32_t col = c0 + c;
    const uint32_t pvc = (uint32_t)__builtin_amdgcn_readlane((int32_t)pv, c);
    bool lose = false;
    for (int k = 0; k < 2 && !lose; ++k) {
      const int32_t x = __builtin_amdgcn_readlane(k ? pw : pu, c);
      const int32_t xb = __builtin_amdgcn_readfirstlane(g.row_ptr[x]);
      const int32_t xd = __builtin_amdgcn_readfirstlane(g.row_ptr[x + 1]) - xb;
      for (int32_t m = 0; m < xd && !lose; m += 64) {
        bool beats = false;
        if (m + lane < xd) {
          const int32_t y = g.col_idx[xb + m + lane];
          const int32_t o = OWN[(int64_t)y * ld + col];
          beats = o >= 0 && o != v && key_beats(0, PRIO[(int64_t)o * ld + col], o, 0, pvc, v);
        }
        lose = __ballot(beats) != 0;
      }
    }
    if (lane == c) win = !lose;
  }
  const unsigned long long bal = __ballot(win);
  if (win && lane == __builtin_ctzll(bal)) *active = 1;
  if (lane < cc) F[e] = win ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_swap_apply_rows(GraphView g, const int8_t *__restrict__ F,
                                                         const int32_t *__restrict__ PU,
                                                         const int32_t *__restrict__ PW, int8_t *__restrict__ Z,
                                                         int32_t *__restrict__ NB, const int32_t *active,
                                                         int32_t ncols, int32_t ld) {
  if (*active == 0) return;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= g.n) return;  // the whole wavefront
  const int32_t lane = threadIdx.x & 63;
  const int32_t c0 = (int32_t)blockIdx.y * 64;
  const int32_t cc = ncols - c0 < 64 ? ncols - c0 : 64;
  const int32_t v = __builtin_amdgcn_readfirstlane((int32_t)(g.lo + row));
  const int64_t e = (int64_t)v * ld + c0 + lane;
  const bool f = lane < cc && F[e] != 0;
  const int32_t pu = f ? PU[e] : -1;
  const int32_t pw = f ? PW[e] : -1;
  unsigned long long wins = __ballot(f);
  while (wins) {
    const int32_t c = __builtin_ctzll(wins);
    wins &= wins - 1;
    const int32_t col = c0 + c;
    const int32_t x3[3] = {v, __builtin_amdgcn_readlane(pu, c), __builtin_amdgcn_readlane(pw, c)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int32_t x = x3[k];
      const int32_t d = k ? 1 : -1;
      if (lane == 0) Z[(int64_t)x * ld + col] = (int8_t)(k ? 1 : 0);
      const int32_t xb = __builtin_amdgcn_readfirstlane(g.row_ptr[x]);
      const int32_t xd = __builtin_amdgcn_readfirstlane(g.row_ptr[x + 1]) - xb;
      for (int32_t m = lane; m < xd; m += 64) atomicAdd(&NB[(int64_t)g.col_idx[xb + m] * ld + col], d);
    }
  }
}

// Total order of 2-flip pairs (gain, (prio_v + prio_u) mod 2^32, -min, -max):
// true iff pair a beats pair b.
__device__ __forceinline__ bool pair_beats(int32_t ga, uint32_t ha, int32_t mina, int32_t maxa, int32_t gb,
                                           uint32_t hb, int32_t minb, int32_t maxb) {
  if (ga != gb) return ga > gb;
  if (ha != hb) return ha > hb;
  if (mina != minb) return mina < minb;
  return maxa < maxb;
}

// Best improving cut edge at v: gain g_v + g_u + 2 w > 0 (g = s t the 1-flip
// gains), largest pair key.  BG = gain, BH = hash, BP = CSR position or -1.
template <bool WEIGHTED>
__global__ __launch_bounds__(256) void k_flip2_best(GraphView g, const int8_t *__restrict__ Z,
                                                    const int32_t *__restrict__ NB, const uint32_t *__restrict__ PRIO,
                                                    int32_t *__restrict__ BG, uint32_t *__restrict__ BH,
                                                    int32_t *__restrict__ BP, int32_t ncols, int32_t ld,
                                                    int32_t lanes_log2) {
  const RowMap m = map_rows<1>(g.n, ncols, lanes_log2);
  if (!m.active) return;
  const int64_t v = g.lo + m.row;
  const int64_t e = v * ld + m.col;
  const int32_t sv = Z[e];
  const int32_t gv = sv * NB[e];
  const uint32_t pv = PRIO[e];
  int32_t bg = 0, bp = -1, bmin = 0, bmax = 0;
  uint32_t bh = 0;
  const int32_t beg = g.row_ptr[v], end = g.row_ptr[v + 1];
  // the neighbours four at a time: their states loaded together, then
  // compared (the best pair key is a maximum, so the order of the
  // comparisons does not change it)
  for (int32_t j0 = beg; j0 < end; j0 += 4) {
    int32_t uq[4], sq[4], nq[4], wq[4];
    uint32_t pq[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) uq[t] = j0 + t < end ? g.col_idx[j0 + t] : -1;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (uq[t] >= 0) {
        const int64_t eu = (int64_t)uq[t] * ld + m.col;
        sq[t] = Z[eu];
        nq[t] = NB[eu];
        pq[t] = PRIO[eu];
        wq[t] = WEIGHTED ? g.weight[j0 + t] : 1;
      } else {
        sq[t] = sv;  // no neighbour: skipped below
        nq[t] = 0;
        pq[t] = 0u;
        wq[t] = 0;
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int32_t u = uq[t], su = sq[t];
      if (u < 0 || su == sv) continue;
      const int32_t gain = gv + su * nq[t] + 2 * wq[t];
      if (gain <= 0) continue;
      const uint32_t h = pv + pq[t];
      const int32_t mn = (int32_t)v < u ? (int32_t)v : u, mx = (int32_t)v < u ? u : (int32_t)v;
      if (bp < 0 || pair_beats(gain, h, mn, mx, bg, bh, bmin, bmax)) {
        bg = gain;
        bh = h;
        bp = j0 + t;
        bmin = mn;
        bmax = mx;
      }
    }
  }
  BG[e] = bg;
  BH[e] = bh;
  BP[e] = bp;
}

// The lower end v of a mutual pair (v, u) applies it (F[v] = 1) when no
// other vertex adjacent to v or u holds a larger best-pair key.
__global__ __launch_bounds__(256) void k_flip2_select(GraphView g, const int32_t *__restrict__ BG,
                                                      const uint32_t *__restrict__ BH,
                                                      const int32_t *__restrict__ BP, int8_t *__restrict__ F,
                                                      int32_t *active, int32_t ncols, int32_t ld,
                                                      int32_t lanes_log2) {
  const RowMap m = map_rows<1>(g.n, ncols, lanes_log2);
  if (!m.active) return;
  const int64_t v = g.lo + m.row;
  const int64_t e = v * ld + m.col;
  const int32_t bp = BP[e];
  bool f = false;
  if (bp >= 0) {
    const int32_t u = g.col_idx[bp];
    const int64_t eu = (int64_t)u * ld + m.col;
    const int32_t bpu = BP[eu];
    if ((int32_t)v < u && bpu >= 0 && g.col_idx[bpu] == (int32_t)v) {
      const int32_t gk = BG[e];
      const uint32_t hk = BH[e];
      f = true;
      for (int k = 0; k < 2 && f; ++k) {
        const int32_t x = k ? u : (int32_t)v;
        const int32_t beg = g.row_ptr[x], end = g.row_ptr[x + 1];
        for (int32_t j = beg; j < end; ++j) {
          const int32_t y = g.col_idx[j];
          if (y == (int32_t)v || y == u) continue;
          const int64_t ey = (int64_t)y * ld + m.col;
          const int32_t bpy = BP[ey];
          if (bpy < 0) continue;
          const int32_t yp = g.col_idx[bpy];
          if (pair_beats(BG[ey], BH[ey], y < yp ? y : yp, y < yp ? yp : y, gk, hk, (int32_t)v, u)) {
            f = false;
            break;
          }
        }
      }
    }
  }
  const unsigned long long bal = __ballot(f);
  if (f && (int)(threadIdx.x & 63) == __builtin_ctzll(bal)) *active = 1;
  F[e] = f ? 1 : 0;
}

template <bool WEIGHTED>
__global__ __launch_bounds__(256) void k_flip2_apply(GraphView g, const int8_t *__restrict__ F,
                                                     const int32_t *__restrict__ BP, int8_t *__restrict__ Z,
                                                     int32_t *__restrict__ NB, const int32_t *active, int32_t ncols,
                                                     int32_t ld, int32_t lanes_log2) {
  if (*active == 0) return;
  const RowMap m = map_rows<1>(g.n, ncols, lanes_log2);
  if (!m.active) return;
  const int64_t v = g.lo + m.row;
  const int64_t e = v * ld + m.col;
  if (!F[e]) return;
  const int32_t x2[2] = {(int32_t)v, g.col_idx[BP[e]]};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int32_t x = x2[k];
    const int64_t ex = (int64_t)x * ld + m.col;
    const int32_t sx = Z[ex];
    Z[ex] = (int8_t)(-sx);
    const int32_t d = -2 * sx;
    const int32_t beg = g.row_ptr[x], end = g.row_ptr[x + 1];
    for (int32_t j = beg; j < end; ++j)
      atomicAdd(&NB[(int64_t)g.col_idx[j] * ld + m.col], WEIGHTED ? d * g.weight[j] : d);
  }
}

// ---------------------------------------------------------------------------
// acceptance: strict improvement, round 0 always (Sec. 4)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_accept_copy(const int8_t *__restrict__ Z, int8_t *__restrict__ Zb,
                                                     const int64_t *__restrict__ value,
                                                     const int64_t *__restrict__ best, int64_t lo, int64_t n,
                                                     int32_t ncols, int32_t ld, int32_t ldb, int32_t first) {
  // one row per lane group of up to 64 lanes, 4 columns per lane when the
  // layout allows 4-byte accesses
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool quad = (ncols & 3) == 0 && (ld & 3) == 0 && (ldb & 3) == 0 && (((uintptr_t)Z | (uintptr_t)Zb) & 3) == 0;
  const int32_t per_row = quad ? ncols >> 2 : ncols;
  if (idx >= n * per_row) return;
  const int64_t v = lo + idx / per_row;
  const int32_t q = (int32_t)(idx % per_row);
  if (quad) {
    const int32_t c = q << 2;
    const uint32_t zq = *reinterpret_cast<const uint32_t *>(Z + v * ld + c);
    uint32_t *dst = reinterpret_cast<uint32_t *>(Zb + v * ldb + c);
    bool take[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) take[i] = first || value[c + i] > best[c + i];
    if (take[0] && take[1] && take[2] && take[3]) {
      *dst = zq;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (take[i]) Zb[v * ldb + c + i] = (int8_t)(zq >> (8 * i));
    }
  } else if (first || value[q] > best[q]) {
    Zb[v * ldb + q] = Z[v * ld + q];
  }
}

__global__ void k_accept_best(const int64_t *__restrict__ value, int64_t *__restrict__ best, int32_t ncols,
                              int32_t first) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  if (first || value[c] > best[c]) best[c] = value[c];
}

// ---------------------------------------------------------------------------
// mutation reset: k smallest (key, v) per column by a 4 x 8-bit radix select
// ---------------------------------------------------------------------------
struct SelState {
  uint32_t prefix, krem, cnteq, tie;
};

__global__ void k_reset_init(SelState *st, uint32_t *hist, int32_t ncols, uint32_t k, uint32_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ncols) st[i] = SelState{0u, k, 0u, n};
  if (i < (int64_t)ncols * 256) hist[i] = 0u;
}

__device__ __forceinline__ uint32_t reset_key(const uint32_t *keys, int64_t lo, int64_t v, int32_t c, int32_t ld,
                                              uint64_t seed, uint64_t traj, uint64_t round) {
  if (keys) return keys[(lo + v) * ld + c];
  return philox_vertex(seed, PURPOSE_RESET, traj, round, (uint64_t)v);
}

// One block per (chunk of RESET_CHUNK rows, column): a 256-bin histogram of
// the current digit in LDS, merged into the column's global histogram with
// one atomic per non-empty bin.
constexpr int64_t RESET_CHUNK = 16384;

__global__ __launch_bounds__(256) void k_reset_hist(const SelState *__restrict__ st, uint32_t *__restrict__ hist,
                                                    const uint32_t *__restrict__ keys, int64_t lo, int64_t n,
                                                    int32_t ld, uint64_t seed, uint64_t traj0, uint64_t round,
                                                    int32_t pass) {
  __shared__ uint32_t sh[256];
  const int32_t c = blockIdx.y;
  sh[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t prefix = st[c].prefix;
  const int hs = 32 - 8 * pass, ds = 24 - 8 * pass;
  const int64_t v0 = (int64_t)blockIdx.x * RESET_CHUNK;
  const int64_t v1 = min(n, v0 + RESET_CHUNK);
  for (int64_t vb = (v0 >> 3) + threadIdx.x; vb * 8 < v1; vb += blockDim.x) {
    uint32_t r[8];
    if (!keys) philox_block8(r, seed, PURPOSE_RESET, traj0 + c, round, (uint64_t)vb);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t v = vb * 8 + i;
      if (v >= v1) break;
      const uint32_t key = keys ? keys[(lo + v) * ld + c] : r[i];
      if (pass == 0 || (key >> hs) == prefix) atomicAdd(&sh[(key >> ds) & 255u], 1u);
    }
  }
  __syncthreads();
  const uint32_t h = sh[threadIdx.x];
  if (h) atomicAdd(&hist[c * 256 + threadIdx.x], h);
}

// one wavefront per column: pick the digit bin holding the krem-th smallest
// key, then clear the column's histogram for the next pass
__global__ __launch_bounds__(64) void k_reset_digit(SelState *st, uint32_t *hist) {
  const int32_t c = blockIdx.x;
  SelState s = st[c];
  uint32_t d, before, at;
  wave_select_digit(hist + c * 256, s.krem, d, before, at);
#pragma unroll
  for (int i = 0; i < 4; ++i) hist[c * 256 + threadIdx.x * 4 + i] = 0u;
  if (threadIdx.x == 0) {
    s.prefix = (s.prefix << 8) | d;
    s.krem -= before;
    s.cnteq = at;
    st[c] = s;
  }
}

// Columns whose threshold key is shared by more vertices than remain to be
// taken keep the lowest indices: tie = largest v taken among equal keys.
__global__ __launch_bounds__(256) void k_reset_ties(SelState *st, const uint32_t *__restrict__ keys, int64_t lo,
                                                    int64_t n, int32_t ld, uint64_t seed, uint64_t traj0,
                                                    uint64_t round) {
  const int32_t c = blockIdx.x;
  __shared__ uint32_t s_cnt[256];
  __shared__ uint32_t s_base;
  __shared__ int32_t s_done;
  SelState s = st[c];
  if (s.cnteq == s.krem) return;  // uniform over the block
  if (threadIdx.x == 0) {
    s_base = 0;
    s_done = 0;
  }
  __syncthreads();
  for (int64_t v0 = 0; v0 < n; v0 += blockDim.x) {
    const int64_t v = v0 + threadIdx.x;
    uint32_t eq = 0;
    if (v < n) eq = reset_key(keys, lo, v, c, ld, seed, traj0 + c, round) == s.prefix ? 1u : 0u;
    s_cnt[threadIdx.x] = eq;
    __syncthreads();
    // inclusive scan (Hillis-Steele)
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
      const uint32_t t = threadIdx.x >= (unsigned)off ? s_cnt[threadIdx.x - off] : 0u;
      __syncthreads();
      s_cnt[threadIdx.x] += t;
      __syncthreads();
    }
    const uint32_t incl = s_base + s_cnt[threadIdx.x];
    if (eq && incl == s.krem) {
      st[c].tie = (uint32_t)v;
      s_done = 1;
    }
    __syncthreads();
    if (s_done) break;
    if (threadIdx.x == blockDim.x - 1) s_base = incl;
    __syncthreads();
  }
}

// base: per column the pool slot to start from (or -1 / nullptr: the
// column's own incumbent in Zb)
template <bool MAXCUT>
__global__ __launch_bounds__(256) void k_reset_apply(const SelState *__restrict__ st, const uint32_t *__restrict__ keys,
                                                     const int8_t *__restrict__ Zb, float *__restrict__ X,
                                                     float *__restrict__ V, int64_t lo, int64_t n, int32_t ncols,
                                                     int32_t ld, int32_t ldb, uint64_t seed, uint64_t traj0,
                                                     uint64_t round, int32_t k, int32_t mode,
                                                     const int8_t *__restrict__ Zp, int32_t ldp,
                                                     const int32_t *__restrict__ base_slot) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nvb = (n + 7) >> 3;
  if (idx >= nvb * ncols) return;
  const int32_t c = (int32_t)(idx % ncols);
  const int64_t vb = idx / ncols;
  uint32_t r[8];
  if (k > 0 && !keys) philox_block8(r, seed, PURPOSE_RESET, traj0 + c, round, (uint64_t)vb);
  SelState s = k > 0 ? st[c] : SelState{0u, 0u, 0u, 0u};
  const int32_t bs = base_slot ? base_slot[c] : -1;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t v = vb * 8 + i;
    if (v >= n) break;
    const float base = (float)(bs >= 0 ? Zp[(lo + v) * ldp + bs] : Zb[(lo + v) * ldb + c]);
    float x = base;
    if (k > 0) {
      const uint32_t key = keys ? keys[(lo + v) * ld + c] : r[i];
      const bool sel = key < s.prefix || (key == s.prefix && (uint32_t)v <= s.tie);
      if (sel) x = mode == 0 ? 0.0f : (MAXCUT ? -base : 1.0f - base);
    }
    X[(lo + v) * ld + c] = x;
    if (V) V[(lo + v) * ld + c] = 0.0f;
  }
}

// ---------------------------------------------------------------------------
// the pmQO pool (Alg. 3 / Alg. 4): top-K distinct solutions per graph
// ---------------------------------------------------------------------------
// SplitMix64 output for state x (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The graph of batch row v: the last g with vtx_off[g] <= v (0 <= v < n_total).
__device__ __forceinline__ int32_t graph_of_row(const int64_t *__restrict__ vtx_off, int32_t G, int64_t v) {
  int32_t lo = 0, hi = G;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (vtx_off[mid] <= v)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// H[g][c] += sum over the rows v of graph g with Z[v][c] > 0 of
// splitmix64(v - lo_g), mod 2^64, for every graph of the batch (H cleared by
// the caller).  Thread per (chunk of 256 batch rows, column): long enough
// that few atomics meet on one column of a large graph; a chunk that runs
// into the next graph adds each part to its own graph.  The additions
// commute, so the sums are exact.
__global__ __launch_bounds__(256) void k_col_hash(const int8_t *__restrict__ Z, const int64_t *__restrict__ vtx_off,
                                                  int32_t G, int64_t n_total, int32_t ncols, int32_t ld,
                                                  unsigned long long *__restrict__ H) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t chunks = (n_total + 255) >> 8;
  if (idx >= chunks * ncols) return;
  const int32_t c = (int32_t)(idx % ncols);
  const int64_t r0 = (idx / ncols) << 8;
  const int64_t r1 = r0 + 256 < n_total ? r0 + 256 : n_total;
  int32_t g = graph_of_row(vtx_off, G, r0);
  int64_t base = vtx_off[g], end = vtx_off[g + 1];
  uint64_t h = 0;
  for (int64_t v = r0; v < r1; ++v) {
    while (v >= end) {
      if (h) atomicAdd(H + (int64_t)g * ncols + c, (unsigned long long)h);
      h = 0;
      ++g;
      base = end;
      end = vtx_off[g + 1];
    }
    if (Z[v * ld + c] > 0) h += splitmix64((uint64_t)(v - base));
  }
  if (h) atomicAdd(H + (int64_t)g * ncols + c, (unsigned long long)h);
}

// One workgroup per graph g = blockIdx.x (taken: K + B bytes per graph).
// Candidates i < K: the old pool's slots (empty
// = INT64_MIN); i >= K: the round's columns (MIS: value -1 = not a
// solution).  K times: the valid, untaken candidate of largest (value,
// -i) fills the next slot, and every candidate with its (value, hash) is
// taken (the union is a set).  SRC[k] = i of slot k or -1.
__global__ __launch_bounds__(256) void k_pool_select(const int64_t *__restrict__ pv_old,
                                                     const unsigned long long *__restrict__ ph_old,
                                                     const int64_t *__restrict__ value,
                                                     const unsigned long long *__restrict__ hash, int32_t K,
                                                     int32_t B, int32_t mis, int8_t *__restrict__ taken,
                                                     int64_t *__restrict__ pv_new,
                                                     unsigned long long *__restrict__ ph_new,
                                                     int32_t *__restrict__ src) {
  __shared__ int64_t sv[4];
  __shared__ int32_t si[4];
  __shared__ int64_t wv;
  __shared__ unsigned long long wh;
  __shared__ int32_t wi;
  const int32_t g = blockIdx.x;
  const int32_t N = K + B;
  pv_old += (int64_t)g * K;
  ph_old += (int64_t)g * K;
  value += (int64_t)g * B;
  hash += (int64_t)g * B;
  taken += (int64_t)g * N;
  auto cand_v = [&](int32_t i) { return i < K ? pv_old[i] : value[i - K]; };
  auto cand_h = [&](int32_t i) { return i < K ? ph_old[i] : hash[i - K]; };
  auto valid = [&](int32_t i) {
    const int64_t v = cand_v(i);
    return i < K ? v != INT64_MIN : !(mis && v < 0);
  };
  for (int32_t i = threadIdx.x; i < N; i += blockDim.x) taken[i] = valid(i) ? 0 : 1;
  __syncthreads();
  for (int32_t k = 0; k < K; ++k) {
    int64_t bv = INT64_MIN;
    int32_t bi = 0x7fffffff;
    for (int32_t i = threadIdx.x; i < N; i += blockDim.x) {
      if (taken[i]) continue;
      const int64_t v = cand_v(i);
      if (bi == 0x7fffffff || v > bv) {  // i ascends within the thread
        bv = v;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const int64_t ov = __shfl_down(bv, off, 64);
      const int32_t oi = __shfl_down(bi, off, 64);
      if (oi != 0x7fffffff && (bi == 0x7fffffff || ov > bv || (ov == bv && oi < bi))) {
        bv = ov;
        bi = oi;
      }
    }
    if ((threadIdx.x & 63) == 0) {
      sv[threadIdx.x >> 6] = bv;
      si[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (si[w] != 0x7fffffff && (bi == 0x7fffffff || sv[w] > bv || (sv[w] == bv && si[w] < bi))) {
          bv = sv[w];
          bi = si[w];
        }
      wi = bi;
      wv = bv;
      if (bi != 0x7fffffff) {
        wh = cand_h(bi);
        pv_new[(int64_t)g * K + k] = bv;
        ph_new[(int64_t)g * K + k] = wh;
        src[(int64_t)g * K + k] = bi;
      } else {
        pv_new[(int64_t)g * K + k] = INT64_MIN;
        ph_new[(int64_t)g * K + k] = 0;
        src[(int64_t)g * K + k] = -1;
      }
    }
    __syncthreads();
    if (wi != 0x7fffffff)
      for (int32_t i = threadIdx.x; i < N; i += blockDim.x)
        if (!taken[i] && cand_v(i) == wv && cand_h(i) == wh) taken[i] = 1;
    __syncthreads();
  }
}

// New pool solutions of every graph: slot k of row v's graph g <- old slot
// SRC[g][k] (< K), column SRC[g][k] - K of Z, or zeros (empty).
__global__ __launch_bounds__(256) void k_pool_copy(const int8_t *__restrict__ pz_old, const int8_t *__restrict__ Z,
                                                   const int32_t *__restrict__ src, int8_t *__restrict__ pz_new,
                                                   const int64_t *__restrict__ vtx_off, int32_t G, int64_t n_total,
                                                   int32_t K, int32_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_total * K) return;
  const int64_t v = idx / K;
  const int32_t k = (int32_t)(idx % K);
  const int32_t s = src[(int64_t)graph_of_row(vtx_off, G, v) * K + k];
  pz_new[v * K + k] = s < 0 ? (int8_t)0 : s < K ? pz_old[v * K + s] : Z[v * ld + (s - K)];
}

// Pool slot each trajectory t = g ncols + c restarts from: (u * size) >> 32,
// u the Philox draw of purpose POOL for (t, round), lane 0, size the filled
// slots of graph g's pool (pv [G][K]); -1 if empty.
__global__ void k_pool_bases(const int64_t *__restrict__ pv, int32_t K, int32_t G, int32_t ncols, uint64_t seed,
                             uint64_t round, int32_t *__restrict__ base) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)G * ncols) return;
  const int64_t *p = pv + (t / ncols) * K;
  int32_t size = 0;
  for (int32_t k = 0; k < K; ++k) size += p[k] != INT64_MIN;
  uint32_t r[8];
  philox_block8(r, seed, PURPOSE_POOL, (uint64_t)t, round, 0);
  base[t] = size ? (int32_t)(((uint64_t)r[0] * (uint64_t)size) >> 32) : -1;
}

// value[k] = INT64_MIN where the pool slot is empty (so a search of an empty
// slot is never accepted)
__global__ void k_mask_empty(int64_t *__restrict__ value, const int64_t *__restrict__ pv, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && pv[i] == INT64_MIN) value[i] = INT64_MIN;
}

// sum of count doubles in a fixed order (one workgroup: lane-strided partial
// sums, then a tree over the 256 lanes), so repeated calls agree bit for bit
__global__ __launch_bounds__(256) void k_sum_f64(const double *__restrict__ in, int64_t count,
                                                 double *__restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) acc += in[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// ---------------------------------------------------------------------------
// best set of the pool modes (I_sol of Alg. 3, S_sol of Alg. 4): graph g is
// offered K candidate values cand[g K + c] in column order and takes each one
// that is strictly above what it holds, so it ends with the first candidate of
// the largest value when that beats sol_v[g].  filled (optional): a candidate
// counts only where filled[g K + c] != INT64_MIN (a pool slot in use);
// need_sol: a graph that holds no set yet (INT64_MIN) takes nothing.
// choice[g] = the column taken, -1 for none.
// ---------------------------------------------------------------------------
__global__ void k_offer_pick(const int64_t *__restrict__ cand, const int64_t *__restrict__ filled, int32_t K,
                             int32_t G, int32_t need_sol, int64_t *__restrict__ sol_v, int32_t *__restrict__ choice) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  int64_t cur = sol_v[g];
  int32_t pick = -1;
  if (!(need_sol && cur == INT64_MIN)) {
    for (int32_t c = 0; c < K; ++c) {
      const int64_t i = (int64_t)g * K + c;
      if (filled && filled[i] == INT64_MIN) continue;
      if (cand[i] > cur) {
        cur = cand[i];
        pick = c;
      }
    }
  }
  choice[g] = pick;
  if (pick >= 0) sol_v[g] = cur;
}

// rows of every graph that took a candidate: sol_z[v] = Z[v ld + choice[g]]
__global__ void k_offer_copy(const int8_t *__restrict__ Z, int32_t ld, const int32_t *__restrict__ choice,
                             const int64_t *__restrict__ voff, int32_t G, int8_t *__restrict__ sol_z, int64_t n_total) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_total) return;
  int32_t lo = 0, hi = G;  // g with voff[g] <= v < voff[g+1]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (voff[mid] <= v)
      lo = mid;
    else
      hi = mid;
  }
  const int32_t c = choice[lo];
  if (c >= 0) sol_z[v] = Z[v * ld + c];
}

// ---------------------------------------------------------------------------
// answer per graph: best incumbent, ties to the lowest trajectory
// ---------------------------------------------------------------------------
// one workgroup per graph: (value, -b) maximised over the trajectories by
// lane strides, a wavefront shuffle tree and the first wavefront
__global__ __launch_bounds__(256) void k_pick_best(const int64_t *__restrict__ best, int32_t G, int32_t B,
                                                   int64_t *__restrict__ best_value, int32_t *__restrict__ best_b) {
  __shared__ int64_t sv[4];
  __shared__ int32_t sb[4];
  const int32_t g = blockIdx.x;
  int64_t bv = INT64_MIN;
  int32_t bb = 0x7fffffff;
  for (int32_t b = threadIdx.x; b < B; b += blockDim.x) {
    const int64_t x = best[(int64_t)g * B + b];
    if (x > bv) {  // b ascends within the thread: ties keep the lower
      bv = x;
      bb = b;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const int64_t ov = __shfl_down(bv, off, 64);
    const int32_t ob = __shfl_down(bb, off, 64);
    if (ov > bv || (ov == bv && ob < bb)) {
      bv = ov;
      bb = ob;
    }
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sv[wave] = bv;
    sb[wave] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (sv[w] > bv || (sv[w] == bv && sb[w] < bb)) {
        bv = sv[w];
        bb = sb[w];
      }
    // nothing but empty pool slots: no answer (-1), slot 0
    best_value[g] = bv == INT64_MIN ? -1 : bv;
    best_b[g] = bb == 0x7fffffff ? 0 : bb;
  }
}

__global__ void k_copy_best_x(const int8_t *__restrict__ Zb, int32_t B, const int64_t *__restrict__ voff, int32_t G,
                              const int32_t *__restrict__ best_b, int8_t *__restrict__ out, int64_t n_total) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_total) return;
  int32_t lo = 0, hi = G;  // find g with voff[g] <= v < voff[g+1]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (voff[mid] <= v)
      lo = mid;
    else
      hi = mid;
  }
  out[v] = Zb[v * B + best_b[lo]];
}

__global__ void k_gather_rowptr(const int32_t *__restrict__ row_ptr, const int64_t *__restrict__ voff, int32_t G,
                                int32_t *__restrict__ out) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g <= G) out[g] = row_ptr[voff[g]];
}

// ---------------------------------------------------------------------------
// graph validation (two phases: row_ptr first, then columns)
// ---------------------------------------------------------------------------
__global__ void k_validate_rows(const int32_t *__restrict__ row_ptr, int64_t n, int64_t nnz, int32_t *err) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v == 0 && (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz)) atomicOr(err, 1);
  if (v < n) {
    const int32_t a = row_ptr[v], b = row_ptr[v + 1];
    if (a > b || a < 0 || (int64_t)b > nnz) atomicOr(err, 1);
  }
}

// Runs in the same pass as k_validate_rows: rows whose row_ptr range is not
// inside [0, nnz] are skipped here (k_validate_rows flags them), so no read
// leaves col_idx.
__global__ void k_validate_cols(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                                const int32_t *__restrict__ weight, const int64_t *__restrict__ voff, int32_t G,
                                int64_t n, int64_t nnz, int32_t *err) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int32_t glo = 0, ghi = G;
  while (ghi - glo > 1) {
    const int32_t mid = (glo + ghi) >> 1;
    if (voff[mid] <= v)
      glo = mid;
    else
      ghi = mid;
  }
  const int64_t lo = voff[glo], hi = voff[glo + 1];
  const int32_t beg = row_ptr[v], end = row_ptr[v + 1];
  if (beg < 0 || beg > end || (int64_t)end > nnz) return;
  int64_t prev = -1;
  for (int32_t j = beg; j < end; ++j) {
    const int64_t c = col_idx[j];
    if (c < lo || c >= hi) {
      atomicOr(err, 2);  // out of the graph's range
      return;
    }
    if (c == v) atomicOr(err, 4);     // self loop
    if (c <= prev) atomicOr(err, 8);  // unsorted or duplicate
    prev = c;
    // symmetry: v must appear in row c (binary search; rows are checked sorted)
    int32_t a = row_ptr[c], b = row_ptr[c + 1] - 1;
    if (a < 0 || a > b + 1 || (int64_t)b >= nnz) continue;  // row c is flagged by the row check
    bool found = false;
    while (a <= b) {
      const int32_t mid = (a + b) >> 1;
      const int64_t x = col_idx[mid];
      if (x == v) {
        found = true;
        if (weight && weight[mid] != weight[j]) atomicOr(err, 32);
        break;
      }
      if (x < v)
        a = mid + 1;
      else
        b = mid - 1;
    }
    if (!found) atomicOr(err, 16);
  }
}

// ---------------------------------------------------------------------------
// differentiation
// ---------------------------------------------------------------------------
// Deterministic per-block column partial sums: val summed over the block's
// rows into part[prow][col .. col+VEC).  Each wavefront first adds its rows
// with a fixed shuffle tree (lanes with equal lane % lanes), then the first
// wavefront adds the per-wave sums in wave order.  Every thread of the block
// must call it; it uses PARTIAL_LDS(VEC) bytes of the dynamic LDS.
#define PARTIAL_LDS(VEC) ((size_t)(256 / 64) * 64 * (VEC) * sizeof(double))

template <int VEC>
__device__ __forceinline__ void block_column_partials(const double (&val)[VEC], bool active, int32_t col,
                                                      int32_t ncols, int32_t lanes_log2, double *part,
                                                      int64_t prow) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  double *s = reinterpret_cast<double *>(dyn_lds);  // [waves][64][VEC]
  const int lanes = 1 << lanes_log2;
  const int wave = threadIdx.x >> 6, wl = threadIdx.x & 63;
  const int nwaves = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < VEC; ++i) {
    double t = active ? val[i] : 0.0;
    for (int off = 32; off >= lanes; off >>= 1) t += __shfl_down(t, off, 64);
    if (wl < lanes) s[(wave * 64 + wl) * VEC + i] = t;
  }
  __syncthreads();
  if (wave == 0 && wl < lanes && col < ncols) {
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      double t = 0.0;
      for (int w = 0; w < nwaves; ++w) t += s[(w * 64 + wl) * VEC + i];
      part[prow * ncols + col + i] = t;
    }
  }
}

// Partials of the objective and gradient of Eq. (3) / (7):
// f_b = sum_v x_v (c + eta/2 (A x)_v), grad = scale_b (c + eta A x).
// Partial rows: one per row workgroup, then one per hub row.
// per-vertex objective contribution (float64): h x (1 - gamma/2 acc),
// f_B x (-lambda - acc), f_A -x acc, f_L x (W x - acc) / 4,
// f_P x (W x - acc + lambda x)
template <int OBJ>
__device__ __forceinline__ void objective_terms(float x, float acc, float W, float param, float sc, float &gr,
                                                double &fv) {
  const float gg = grad_of<OBJ>(acc, x, W, param);
  gr = sc * gg;
  const double xd = x, ad = acc;
  if constexpr (OBJ == OBJ_H) {
    fv = xd * (1.0 - 0.5 * (double)param * ad);
  } else if constexpr (OBJ == OBJ_FB) {
    fv = xd * (-(double)param - ad);
  } else if constexpr (OBJ == OBJ_FA) {
    fv = -xd * ad;
  } else if constexpr (OBJ == OBJ_FL) {
    fv = 0.25 * xd * ((double)W * xd - ad);
  } else {
    fv = xd * ((double)W * xd - ad + (double)param * xd);
  }
}

template <int VEC, int OBJ, bool WEIGHTED, int ROWS, int KB = 4>
__global__ __launch_bounds__(256) void k_objective_grad(GraphView g, const float *__restrict__ X,
                                                        const float *__restrict__ scale, float *__restrict__ grad,
                                                        double *__restrict__ part, int32_t ncols, int32_t ld,
                                                        int32_t lanes_log2, float param) {
  const int64_t nhb = hub_blocks(g, ncols);
  const int64_t nrb = gridDim.x - nhb;  // row workgroups
  const Blk blk = xcd_blk(g.xcd_local);
  if (blk.x < nhb) {
    if (blk.y != 0) return;
    const HubItem it = hub_item(g, ncols, blk.x);
    const float acc = hub_gather<WEIGHTED>(g, X, it, ld);
    if ((int32_t)threadIdx.x < it.cw) {
      const int32_t c = it.c0 + threadIdx.x;
      const int64_t e = it.v * ld + c;
      float gr;
      double fv;
      const float W = OBJ == OBJ_FL || OBJ == OBJ_FP ? weighted_degree<WEIGHTED>(g, it.v) : 0.0f;
      objective_terms<OBJ>(X[e], acc, W, param, scale ? scale[c] : 1.0f, gr, fv);
      if (grad) grad[e] = gr;
      if (part) part[(nrb + it.h) * ncols + c] = fv;
    }
    return;
  }
  int64_t v[ROWS];
  bool own[ROWS];
  int32_t col;
  float acc[ROWS][VEC];
  int32_t wsum[ROWS];
  group_gather<VEC, WEIGHTED, ROWS, KB>(g, X, blk.x - nhb, blk.y, ncols, ld, lanes_log2, v, own, col, acc, wsum);
  double fv[VEC];
#pragma unroll
  for (int i = 0; i < VEC; ++i) fv[i] = 0.0;
  bool any = false;
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    if (!own[k] || col >= ncols) continue;
    any = true;
    float x[VEC], gr[VEC];
    load_vec<VEC>(X + v[k] * ld + col, x);
    const float W = OBJ == OBJ_FL || OBJ == OBJ_FP ? (float)wsum[k] : 0.0f;
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      double f;
      objective_terms<OBJ>(x[i], acc[k][i], W, param, scale ? scale[col + i] : 1.0f, gr[i], f);
      fv[i] += f;
    }
    if (grad) store_vec<VEC>(grad + v[k] * ld + col, gr);
  }
  if (part) block_column_partials<VEC>(fv, any, col, ncols, lanes_log2, part, blk.x - nhb);
}

// Column sums of per-block partials part[nblk][ncols] in a fixed order.
// Block (x, y) sums, for W = 2^wlog2 consecutive columns, the partial rows
// [y * per_slice, (y + 1) * per_slice): lane group r of the block takes rows
// r, r + R, ... (R = 256 / W; coalesced over the columns), then a fixed tree
// over r.  With gridDim.y > 1 it writes dst[y][ncols] (the next level);
// with one slice it writes (or adds to) the final dst[ncols].
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ part, int64_t nblk, int32_t ncols,
                                                         int32_t wlog2, int64_t per_slice, double *__restrict__ dst,
                                                         int32_t accumulate) {
  __shared__ double s[256];
  const int32_t W = 1 << wlog2, R = 256 >> wlog2;
  const int32_t c = blockIdx.x * W + (threadIdx.x & (W - 1));
  const int32_t r = threadIdx.x >> wlog2;
  const int64_t b0 = (int64_t)blockIdx.y * per_slice;
  const int64_t b1 = min(nblk, b0 + per_slice);
  double t = 0.0;
  if (c < ncols) {
#pragma unroll 8
    for (int64_t b = b0 + r; b < b1; b += R) t += part[b * ncols + c];
  }
  s[threadIdx.x] = t;
  __syncthreads();
  for (int32_t off = R >> 1; off > 0; off >>= 1) {
    if (r < off) s[threadIdx.x] += s[threadIdx.x + (off << wlog2)];
    __syncthreads();
  }
  if (r == 0 && c < ncols) {
    if (gridDim.y > 1)
      dst[(int64_t)blockIdx.y * ncols + c] = s[threadIdx.x];
    else
      dst[c] = accumulate ? dst[c] + s[threadIdx.x] : s[threadIdx.x];
  }
}

// adjoint, part 1: recompute g(x_k), the clip mask, mu = mask * lam_next,
// and partials of <mu, g> for dL/dalpha (rows as in k_objective_grad)
template <int OBJ>
__device__ __forceinline__ void adjoint_mu(float x, float ln, float acc, float W, float alpha, float param, float &mu,
                                           double &dv) {
  constexpr bool MAXCUT = OBJ != OBJ_H;
  const float gr = grad_of<OBJ>(acc, x, W, param);
  const float s = alpha * gr;
  const float z = x + s;
  const bool mask = z >= box_lo<MAXCUT>() && z <= box_hi();
  mu = mask ? ln : 0.0f;
  dv = (double)mu * (double)gr;
}

template <int VEC, int OBJ, bool WEIGHTED, int ROWS, int KB = 4>
__global__ __launch_bounds__(256) void k_adj_mu(GraphView g, const float *__restrict__ Xk,
                                                const float *__restrict__ lam_next, float *__restrict__ mu_out,
                                                double *__restrict__ part, int32_t ncols, int32_t ld,
                                                int32_t lanes_log2, float alpha, float param) {
  const int64_t nhb = hub_blocks(g, ncols);
  const int64_t nrb = gridDim.x - nhb;
  const Blk blk = xcd_blk(g.xcd_local);
  if (blk.x < nhb) {
    if (blk.y != 0) return;
    const HubItem it = hub_item(g, ncols, blk.x);
    const float acc = hub_gather<WEIGHTED>(g, Xk, it, ld);
    if ((int32_t)threadIdx.x < it.cw) {
      const int32_t c = it.c0 + threadIdx.x;
      const int64_t e = it.v * ld + c;
      float mu;
      double dv;
      const float W = OBJ == OBJ_FL || OBJ == OBJ_FP ? weighted_degree<WEIGHTED>(g, it.v) : 0.0f;
      adjoint_mu<OBJ>(Xk[e], lam_next[e], acc, W, alpha, param, mu, dv);
      mu_out[e] = mu;
      part[(nrb + it.h) * ncols + c] = dv;
    }
    return;
  }
  int64_t v[ROWS];
  bool own[ROWS];
  int32_t col;
  float acc[ROWS][VEC];
  int32_t wsum[ROWS];
  group_gather<VEC, WEIGHTED, ROWS, KB>(g, Xk, blk.x - nhb, blk.y, ncols, ld, lanes_log2, v, own, col, acc, wsum);
  double dv[VEC];
#pragma unroll
  for (int i = 0; i < VEC; ++i) dv[i] = 0.0;
  bool any = false;
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    if (!own[k] || col >= ncols) continue;
    any = true;
    float x[VEC], ln[VEC], mu[VEC];
    load_vec<VEC>(Xk + v[k] * ld + col, x);
    load_vec<VEC>(lam_next + v[k] * ld + col, ln);
    const float W = OBJ == OBJ_FL || OBJ == OBJ_FP ? (float)wsum[k] : 0.0f;
#pragma unroll
    for (int i = 0; i < VEC; ++i) {
      double d;
      adjoint_mu<OBJ>(x[i], ln[i], acc[k][i], W, alpha, param, mu[i], d);
      dv[i] += d;
    }
    store_vec<VEC>(mu_out + v[k] * ld + col, mu);
  }
  block_column_partials<VEC>(dv, any, col, ncols, lanes_log2, part, blk.x - nhb);
}

// adjoint, part 2: lam_k = mu + alpha (H mu), H the objective's Hessian:
// -gamma A (h), -2 A (f_B, f_A), (D - A) / 2 (f_L), 2 (D - A + lambda I) (f_P)
template <int OBJ>
__device__ __forceinline__ float adjoint_lambda(float mv, float acc, float W, float alpha, float param) {
  float hm;
  if constexpr (OBJ == OBJ_H) {
    hm = (-param) * acc;
  } else if constexpr (OBJ == OBJ_FB || OBJ == OBJ_FA) {
    hm = -2.0f * acc;
  } else {
    const float t1 = W * mv;
    const float t2 = t1 - acc;
    if constexpr (OBJ == OBJ_FL) {
      hm = 0.5f * t2;
    } else {
      const float t3 = param * mv;
      const float t4 = t2 + t3;
      hm = 2.0f * t4;
    }
  }
  const float t = alpha * hm;
  return mv + t;
}

template <int VEC, int OBJ, bool WEIGHTED, int ROWS, int KB = 4>
__global__ __launch_bounds__(256) void k_adj_lambda(GraphView g, const float *__restrict__ mu, float *__restrict__ lam,
                                                    int32_t ncols, int32_t ld, int32_t lanes_log2, float alpha,
                                                    float param) {
  const int64_t nhb = hub_blocks(g, ncols);
  const Blk blk = xcd_blk(g.xcd_local);
  if (blk.x < nhb) {
    if (blk.y != 0) return;
    const HubItem it = hub_item(g, ncols, blk.x);
    const float acc = hub_gather<WEIGHTED>(g, mu, it, ld);
    if ((int32_t)threadIdx.x < it.cw) {
      const int64_t e = it.v * ld + it.c0 + threadIdx.x;
      const float W = OBJ == OBJ_FL || OBJ == OBJ_FP ? weighted_degree<WEIGHTED>(g, it.v) : 0.0f;
      lam[e] = adjoint_lambda<OBJ>(mu[e], acc, W, alpha, param);
    }
    return;
  }
  int64_t v[ROWS];
  bool own[ROWS];
  int32_t col;
  float acc[ROWS][VEC];
  int32_t wsum[ROWS];
  group_gather<VEC, WEIGHTED, ROWS, KB>(g, mu, blk.x - nhb, blk.y, ncols, ld, lanes_log2, v, own, col, acc, wsum);
  if (col >= ncols) return;
#pragma unroll
  for (int k = 0; k < ROWS; ++k) {
    if (!own[k]) continue;
    float mv[VEC], out[VEC];
    load_vec<VEC>(mu + v[k] * ld + col, mv);
    const float W = OBJ == OBJ_FL || OBJ == OBJ_FP ? (float)wsum[k] : 0.0f;
#pragma unroll
    for (int i = 0; i < VEC; ++i) out[i] = adjoint_lambda<OBJ>(mv[i], acc[k][i], W, alpha, param);
    store_vec<VEC>(lam + v[k] * ld + col, out);
  }
}

// ===========================================================================
// host launchers
// ===========================================================================
#define MQO_LAUNCH(kernel, grid, block, shmem, stream, ...) \
  hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__)

static inline unsigned blocks_for(int64_t count, int threads = 256) {
  int64_t b = (count + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > 2147483647LL) b = 2147483647LL;
  return (unsigned)b;
}

void launch_init_uniform(bool maxcut, float *X, int64_t lo, int64_t n, int32_t ncols, int32_t ld, uint64_t seed,
                         uint64_t traj0, hipStream_t s, uint64_t start) {
  const int64_t count = ((n + 7) >> 3) * ncols;
  if (maxcut)
    MQO_LAUNCH(k_init_uniform<true>, dim3(blocks_for(count)), dim3(256), 0, s, X, lo, n, ncols, ld, seed, traj0,
               start);
  else
    MQO_LAUNCH(k_init_uniform<false>, dim3(blocks_for(count)), dim3(256), 0, s, X, lo, n, ncols, ld, seed, traj0,
               start);
}

void launch_degree_max(const int32_t *row_ptr, int64_t n, int32_t *out, hipStream_t s) {
  MQO_LAUNCH(k_fill_i32, dim3(1), dim3(64), 0, s, out, (int64_t)1, 0);
  MQO_LAUNCH(k_degree_max, dim3(blocks_for(n < 262144 ? n : 262144)), dim3(256), 0, s, row_ptr, (int64_t)0, n, out);
}

void launch_init_degree(bool maxcut, float *X, const int32_t *row_ptr, int32_t *dmax_scratch, int64_t lo, int64_t n,
                        int32_t ncols, int32_t ld, uint64_t seed, uint64_t traj0, float sigma, hipStream_t s,
                        uint64_t start) {
  MQO_LAUNCH(k_fill_i32, dim3(1), dim3(64), 0, s, dmax_scratch, (int64_t)1, 0);
  MQO_LAUNCH(k_degree_max, dim3(blocks_for(n < 65536 ? n : 65536)), dim3(256), 0, s, row_ptr, lo, n, dmax_scratch);
  const int64_t count = n * ncols;
  if (maxcut)
    MQO_LAUNCH(k_init_degree<true>, dim3(blocks_for(count)), dim3(256), 0, s, X, row_ptr, dmax_scratch, lo, n, ncols,
               ld, seed, traj0, sigma, start);
  else
    MQO_LAUNCH(k_init_degree<false>, dim3(blocks_for(count)), dim3(256), 0, s, X, row_ptr, dmax_scratch, lo, n,
               ncols, ld, seed, traj0, sigma, start);
}

StepCfg default_step_cfg(int32_t ncols, int32_t ld) {
  StepCfg c;
  c.vec = 1;
  if (ncols % 4 == 0 && ld % 4 == 0 && ncols >= 16)
    c.vec = 4;
  else if (ncols % 2 == 0 && ld % 2 == 0 && ncols >= 8)
    c.vec = 2;
  c.lanes_log2 = lanes_log2_for((ncols + c.vec - 1) / c.vec);
  return c;
}

// Row workgroups of a sparse-product kernel plus, in front, one workgroup per
// (hub row, column slice).
// rows per lane group of the sparse-product kernels: pairs on near-regular
// graphs when a row has 4 or more lanes (the lockstep gather shuffles
// indices)
static inline int spmm_rows(const GraphView &g, int ll) { return g.pairs && ll >= 2 ? 2 : 1; }

static inline dim3 spmm_grid(const GraphView &g, int32_t ncols, int ll, int vec) {
  const int rows = spmm_rows(g, ll);
  dim3 grid = grid_rows((g.n + rows - 1) / rows, ncols, ll, vec, 256);
  grid.x = (unsigned)(grid.x + hub_blocks(g, ncols));
  return grid;
}

// Calls F::template run<OBJ, WEIGHTED>(args...) for the launch's objective
// form and weights: MIS only unweighted, every MaxCut formulation either.
template <typename F, typename... Args>
static void dispatch_form(int form, bool weighted, Args &&...args) {
  switch (form) {
    case OBJ_H:
      F::template run<OBJ_H, false>(args...);
      break;
    case OBJ_FB:
      if (weighted) F::template run<OBJ_FB, true>(args...);
      else F::template run<OBJ_FB, false>(args...);
      break;
    case OBJ_FL:
      if (weighted) F::template run<OBJ_FL, true>(args...);
      else F::template run<OBJ_FL, false>(args...);
      break;
    case OBJ_FP:
      if (weighted) F::template run<OBJ_FP, true>(args...);
      else F::template run<OBJ_FP, false>(args...);
      break;
    default:
      if (weighted) F::template run<OBJ_FA, true>(args...);
      else F::template run<OBJ_FA, false>(args...);
      break;
  }
}

template <int VEC, bool MOMENTUM>
struct StepLaunch {
  template <int OBJ, bool W>
  static void run(const GraphView &g, const float *X, float *Xn, float *V, int32_t ncols, int32_t ld, int ll,
                  float alpha, float mu, float param, const int8_t *colact, hipStream_t s) {
    const size_t lds = g.nhub ? hub_lds(W) : 0;
    const dim3 grid = spmm_grid(g, ncols, ll, VEC);
    if (spmm_rows(g, ll) == 2) {
      MQO_LAUNCH((k_pga_step<VEC, OBJ, W, MOMENTUM, 2>), grid, dim3(256), lds, s, g, X, Xn, V, ncols, ld, ll, alpha, mu,
                 param, colact);
      return;
    }
    if (g.nhub > 0)  // uneven degrees: eight gathers in flight per lane group
      MQO_LAUNCH((k_pga_step<VEC, OBJ, W, MOMENTUM, 1, 8>), grid, dim3(256), lds, s, g, X, Xn, V, ncols, ld, ll,
                 alpha, mu, param, colact);
    else
      MQO_LAUNCH((k_pga_step<VEC, OBJ, W, MOMENTUM, 1>), grid, dim3(256), lds, s, g, X, Xn, V, ncols, ld, ll, alpha,
                 mu, param, colact);
  }
};

void launch_pga_step(int form, const GraphView &g, const float *X, float *Xn, float *V, int32_t ncols, int32_t ld,
                     StepCfg cfg, float alpha, float mu, float param, hipStream_t s, const int8_t *colact) {
  const bool w = g.weight != nullptr, m = mu != 0.0f;
  const int ll = cfg.lanes_log2;
#define MQO_STEP(VV)                                                                                              \
  if (m)                                                                                                         \
    dispatch_form<StepLaunch<VV, true>>(form, w, g, X, Xn, V, ncols, ld, ll, alpha, mu, param, colact, s);   \
  else                                                                                                           \
    dispatch_form<StepLaunch<VV, false>>(form, w, g, X, Xn, V, ncols, ld, ll, alpha, mu, param, colact, s);
  if (cfg.vec == 4) {
    MQO_STEP(4)
  } else if (cfg.vec == 2) {
    MQO_STEP(2)
  } else {
    MQO_STEP(1)
  }
#undef MQO_STEP
}

void launch_copy_f32(const float *a, float *b, int64_t count, hipStream_t s) {
  MQO_LAUNCH(k_copy_f32, dim3(blocks_for(count < (1 << 24) ? count : (1 << 24))), dim3(256), 0, s, a, b, count);
}

void launch_strided_copy_f32(const float *src, int32_t lds, int32_t cs, float *dst, int32_t ldd, int32_t cd,
                             int64_t lo, int64_t n, hipStream_t s) {
  MQO_LAUNCH(k_strided_copy_f32, dim3(blocks_for(n)), dim3(256), 0, s, src, lds, cs, dst, ldd, cd, lo, n);
}

// early exit: trajectories whose rounded point is fixed stop stepping
__global__ void k_active_update(int8_t *__restrict__ colact, const int8_t *__restrict__ fixed, int32_t ncols) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols && fixed[c]) colact[c] = 0;
}

// executed-step counters: + len for every active trajectory
__global__ void k_count_steps(const int8_t *__restrict__ colact, int64_t *__restrict__ steps, int32_t ncols,
                              int32_t len) {
  const int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols && colact[c]) steps[c] += len;
}

__global__ void k_fill_i8(int8_t *p, int64_t count, int8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_add_i64(int64_t *p, int64_t count, int64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] += v;
}

// out += sum over trajectories t = g*B + b of steps[t] * nnz_g, nnz_g from
// the row_ptr entries at the graph boundaries (rpat[G+1]); out zeroed first
__global__ void k_edge_updates(const int64_t *__restrict__ steps, const int32_t *__restrict__ rpat, int32_t G,
                               int32_t B, unsigned long long *out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = 0;
  if (t < (int64_t)G * B) {
    const int32_t g = (int32_t)(t / B);
    v = (unsigned long long)steps[t] * (unsigned long long)(rpat[g + 1] - rpat[g]);
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

void launch_fill_i8(int8_t *p, int64_t count, int8_t v, hipStream_t s) {
  MQO_LAUNCH(k_fill_i8, dim3(blocks_for(count < 262144 ? count : 262144)), dim3(256), 0, s, p, count, v);
}

void launch_add_i64(int64_t *p, int64_t count, int64_t v, hipStream_t s) {
  MQO_LAUNCH(k_add_i64, dim3(blocks_for(count < 262144 ? count : 262144)), dim3(256), 0, s, p, count, v);
}

void launch_edge_updates(const int64_t *steps, const int32_t *rpat, int32_t G, int32_t B, int64_t *out,
                         hipStream_t s) {
  launch_fill_i64(out, 1, 0, s);
  MQO_LAUNCH(k_edge_updates, dim3(blocks_for((int64_t)G * B)), dim3(256), 0, s, steps, rpat, G, B,
             reinterpret_cast<unsigned long long *>(out));
}

void launch_active_update(int8_t *colact, const int8_t *fixed, int32_t ncols, hipStream_t s) {
  MQO_LAUNCH(k_active_update, dim3(blocks_for(ncols)), dim3(256), 0, s, colact, fixed, ncols);
}

void launch_count_steps(const int8_t *colact, int64_t *steps, int32_t ncols, int32_t len, hipStream_t s) {
  MQO_LAUNCH(k_count_steps, dim3(blocks_for(ncols)), dim3(256), 0, s, colact, steps, ncols, len);
}

void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s) {
  MQO_LAUNCH(k_fill_i32, dim3(blocks_for(count < (1 << 24) ? count : (1 << 24))), dim3(256), 0, s, p, count, v);
}

void launch_fill_i64(int64_t *p, int64_t count, int64_t v, hipStream_t s) {
  MQO_LAUNCH(k_fill_i64, dim3(blocks_for(count < (1 << 24) ? count : (1 << 24))), dim3(256), 0, s, p, count, v);
}

void launch_fill_f32(float *p, int64_t count, float v, hipStream_t s) {
  MQO_LAUNCH(k_fill_f32, dim3(blocks_for(count < (1 << 24) ? count : (1 << 24))), dim3(256), 0, s, p, count, v);
}

void launch_round(bool maxcut, const float *X, int8_t *Z, int64_t lo, int64_t n, int32_t ncols, int32_t ld,
                  hipStream_t s) {
  const int64_t count = n * ncols;
  if (maxcut)
    MQO_LAUNCH(k_round<true>, dim3(blocks_for(count)), dim3(256), 0, s, X, Z, lo, n, ncols, ld);
  else
    MQO_LAUNCH(k_round<false>, dim3(blocks_for(count)), dim3(256), 0, s, X, Z, lo, n, ncols, ld);
}

void launch_evaluate(bool maxcut, const GraphView &g, const int8_t *Z, int32_t *NB, long long *acc, int64_t *value,
                     int64_t *conflicts, int8_t *fixed, int32_t ncols, int32_t ld, hipStream_t s) {
  launch_fill_i64(reinterpret_cast<int64_t *>(acc), 3LL * ncols, 0, s);
  // four columns per lane where the rows of Z and NB allow 4- and 16-byte access
  const bool v4 = ncols % 4 == 0 && ld % 4 == 0 && ((uintptr_t)Z & 3) == 0 && ((uintptr_t)NB & 15) == 0;
  const int vec = v4 ? 4 : 1;
  const int ll = lanes_log2_for(ncols / vec);
  dim3 grid = grid_rows(g.n, ncols, ll, vec, 256);
  if (grid.x > 2048) grid.x = 2048;  // workgroups stride over the rows
  unsigned long long *a = reinterpret_cast<unsigned long long *>(acc);
  const bool w = g.weight != nullptr;
#define MQO_EVAL(MC, W)                                                                          \
  if (v4)                                                                                        \
    MQO_LAUNCH((k_nbr_eval<MC, W, 4>), grid, dim3(256), 0, s, g, Z, NB, a, ncols, ld, ll);       \
  else                                                                                           \
    MQO_LAUNCH((k_nbr_eval<MC, W, 1>), grid, dim3(256), 0, s, g, Z, NB, a, ncols, ld, ll);
  if (maxcut) {
    if (w) {
      MQO_EVAL(true, true)
    } else {
      MQO_EVAL(true, false)
    }
    MQO_LAUNCH(k_value_finalize<true>, dim3(blocks_for(ncols)), dim3(256), 0, s, acc, ncols, value, conflicts,
               fixed);
  } else {
    MQO_EVAL(false, false)
    MQO_LAUNCH(k_value_finalize<false>, dim3(blocks_for(ncols)), dim3(256), 0, s, acc, ncols, value, conflicts,
               fixed);
  }
#undef MQO_EVAL
}

void launch_ls_prio(uint32_t *PRIO, int64_t lo, int64_t n, int32_t ncols, int32_t ld, uint64_t seed, uint64_t traj0,
                    uint64_t round, hipStream_t s) {
  const int64_t count = ((n + 7) >> 3) * ncols;
  MQO_LAUNCH(k_ls_prio, dim3(blocks_for(count)), dim3(256), 0, s, PRIO, lo, n, ncols, ld, seed, traj0, round,
             (uint64_t)PURPOSE_LS);
}

void launch_swap_prio(uint32_t *PRIO, int64_t lo, int64_t n, int32_t ncols, int32_t ld, uint64_t seed,
                      uint64_t traj0, uint64_t round, hipStream_t s) {
  const int64_t count = ((n + 7) >> 3) * ncols;
  MQO_LAUNCH(k_ls_prio, dim3(blocks_for(count)), dim3(256), 0, s, PRIO, lo, n, ncols, ld, seed, traj0, round,
             (uint64_t)PURPOSE_SWAP);
}

void launch_pair_candidates(bool maxcut, const GraphView &g, const int8_t *Z, const int32_t *NB,
                            const uint32_t *PRIO, int32_t *T0, int32_t *T1, int32_t *T2, uint32_t *TB, int32_t ncols,
                            int32_t ld, double mean_degree, hipStream_t s) {
  const int ll = lanes_log2_for(ncols);
  const dim3 grid = grid_rows(g.n, ncols, ll, 1, 256);
  if (maxcut) {
    if (g.weight)
      MQO_LAUNCH(k_flip2_best<true>, grid, dim3(256), 0, s, g, Z, NB, PRIO, T0, reinterpret_cast<uint32_t *>(T1), T2,
                 ncols, ld, ll);
    else
      MQO_LAUNCH(k_flip2_best<false>, grid, dim3(256), 0, s, g, Z, NB, PRIO, T0, reinterpret_cast<uint32_t *>(T1),
                 T2, ncols, ld, ll);
  } else {
    // owners of the proposed insertions, -1 elsewhere
    MQO_LAUNCH(k_fill_rows_i32, grid, dim3(256), 0, s, T2, g.lo, g.n, -1, ncols, ld, ll);
    // one wavefront per (row, 64 columns)
    const dim3 wgrid = grid_rows(g.n, ncols, 6, 1, 256);
    unsigned long long *tb = reinterpret_cast<unsigned long long *>(TB);
    MQO_LAUNCH(k_tight_bits, wgrid, dim3(256), 0, s, g, Z, NB, tb, ncols, ld);
    if (mean_degree >= 24.0)
      MQO_LAUNCH(k_swap_propose, wgrid, dim3(256), 0, s, g, Z, tb, T0, T1, T2, ncols, ld);
    else
      MQO_LAUNCH(k_swap_propose_lanes, grid, dim3(256), 0, s, g, Z, tb, T0, T1, T2, ncols, ld, ll);
  }
}

void launch_pair_apply(bool maxcut, const GraphView &g, int8_t *Z, int32_t *NB, const uint32_t *PRIO, int8_t *F,
                       const int32_t *T0, const int32_t *T1, const int32_t *T2, int32_t *active, int32_t ncols,
                       int32_t ld, double mean_degree, hipStream_t s) {
  const int ll = lanes_log2_for(ncols);
  const dim3 grid = grid_rows(g.n, ncols, ll, 1, 256);
  if (maxcut) {
    MQO_LAUNCH(k_flip2_select, grid, dim3(256), 0, s, g, T0, reinterpret_cast<const uint32_t *>(T1), T2, F, active,
               ncols, ld, ll);
    if (g.weight)
      MQO_LAUNCH(k_flip2_apply<true>, grid, dim3(256), 0, s, g, F, T2, Z, NB, active, ncols, ld, ll);
    else
      MQO_LAUNCH(k_flip2_apply<false>, grid, dim3(256), 0, s, g, F, T2, Z, NB, active, ncols, ld, ll);
  } else {
    if (mean_degree >= 24.0) {
      const dim3 wgrid = grid_rows(g.n, ncols, 6, 1, 256);  // one wavefront per (row, 64 columns)
      MQO_LAUNCH(k_swap_select_rows, wgrid, dim3(256), 0, s, g, T0, T1, T2, PRIO, F, active, ncols, ld);
      MQO_LAUNCH(k_swap_apply_rows, wgrid, dim3(256), 0, s, g, F, T0, T1, Z, NB, active, ncols, ld);
    } else {
      MQO_LAUNCH(k_swap_select, grid, dim3(256), 0, s, g, T0, T1, T2, PRIO, F, active, ncols, ld, ll);
      MQO_LAUNCH(k_swap_apply, grid, dim3(256), 0, s, g, F, T0, T1, Z, NB, active, ncols, ld, ll);
    }
  }
}

void launch_ls_iteration(bool maxcut, const GraphView &g, int8_t *Z, int32_t *NB, const uint32_t *PRIO, int8_t *F,
                         int32_t *active, const int32_t *prev_active, int32_t ncols, int32_t ld, double mean_degree,
                         hipStream_t s) {
  const int ll = lanes_log2_for(ncols);
  const dim3 grid = grid_rows(g.n, ncols, ll, 1, 256);
  const bool w = g.weight != nullptr;
  if (mean_degree >= 24.0) {
    const dim3 wgrid = grid_rows(g.n, ncols, 6, 1, 256);  // one wavefront per (row, 64 columns)
    if (maxcut) {
      MQO_LAUNCH(k_ls_select_rows<true>, wgrid, dim3(256), 0, s, g, Z, NB, PRIO, F, active, prev_active, ncols, ld);
      if (w)
        MQO_LAUNCH((k_ls_apply_rows<true, true>), wgrid, dim3(256), 0, s, g, F, Z, NB, active, ncols, ld);
      else
        MQO_LAUNCH((k_ls_apply_rows<true, false>), wgrid, dim3(256), 0, s, g, F, Z, NB, active, ncols, ld);
    } else {
      MQO_LAUNCH(k_ls_select_rows<false>, wgrid, dim3(256), 0, s, g, Z, NB, PRIO, F, active, prev_active, ncols, ld);
      MQO_LAUNCH((k_ls_apply_rows<false, false>), wgrid, dim3(256), 0, s, g, F, Z, NB, active, ncols, ld);
    }
    return;
  }
  if (maxcut) {
    MQO_LAUNCH(k_ls_select<true>, grid, dim3(256), 0, s, g, Z, NB, PRIO, F, active, prev_active, ncols, ld, ll);
    if (w)
      MQO_LAUNCH((k_ls_apply<true, true>), grid, dim3(256), 0, s, g, F, Z, NB, active, ncols, ld, ll);
    else
      MQO_LAUNCH((k_ls_apply<true, false>), grid, dim3(256), 0, s, g, F, Z, NB, active, ncols, ld, ll);
  } else {
    MQO_LAUNCH(k_ls_select<false>, grid, dim3(256), 0, s, g, Z, NB, PRIO, F, active, prev_active, ncols, ld, ll);
    MQO_LAUNCH((k_ls_apply<false, false>), grid, dim3(256), 0, s, g, F, Z, NB, active, ncols, ld, ll);
  }
}

void launch_accept(const int8_t *Z, int8_t *Zb, const int64_t *value, int64_t *best, int64_t lo, int64_t n,
                   int32_t ncols, int32_t ld, int32_t ldb, bool first, hipStream_t s) {
  const bool quad = (ncols & 3) == 0 && (ld & 3) == 0 && (ldb & 3) == 0 && (((uintptr_t)Z | (uintptr_t)Zb) & 3) == 0;
  MQO_LAUNCH(k_accept_copy, dim3(blocks_for(n * (quad ? ncols >> 2 : ncols))), dim3(256), 0, s, Z, Zb, value, best, lo,
             n, ncols, ld, ldb, (int32_t)first);
  MQO_LAUNCH(k_accept_best, dim3(blocks_for(ncols)), dim3(256), 0, s, value, best, ncols, (int32_t)first);
}

size_t reset_scratch_bytes(int32_t ncols) { return (size_t)ncols * (sizeof(SelState) + 256 * sizeof(uint32_t)); }

void launch_reset(bool maxcut, const int8_t *Zb, int32_t ldb, const uint32_t *keys, float *X, float *V, int64_t lo,
                  int64_t n, int32_t ncols, int32_t ld, uint64_t seed, uint64_t traj0, uint64_t round, int32_t k,
                  int32_t mode, void *scratch, hipStream_t s, const int8_t *Zp, int32_t ldp, const int32_t *base_slot) {
  SelState *st = reinterpret_cast<SelState *>(scratch);
  uint32_t *hist = reinterpret_cast<uint32_t *>(st + ncols);
  const int64_t cnt = ((n + 7) >> 3) * ncols;
  if (k > 0) {
    MQO_LAUNCH(k_reset_init, dim3(blocks_for((int64_t)ncols * 256)), dim3(256), 0, s, st, hist, ncols, (uint32_t)k,
               (uint32_t)n);
    const dim3 hgrid((unsigned)((n + RESET_CHUNK - 1) / RESET_CHUNK), (unsigned)ncols);
    for (int pass = 0; pass < 4; ++pass) {
      MQO_LAUNCH(k_reset_hist, hgrid, dim3(256), 0, s, st, hist, keys, lo, n, ld, seed, traj0, round, pass);
      MQO_LAUNCH(k_reset_digit, dim3(ncols), dim3(64), 0, s, st, hist);
    }
    MQO_LAUNCH(k_reset_ties, dim3(ncols), dim3(256), 0, s, st, keys, lo, n, ld, seed, traj0, round);
  }
  if (maxcut)
    MQO_LAUNCH(k_reset_apply<true>, dim3(blocks_for(cnt)), dim3(256), 0, s, st, keys, Zb, X, V, lo, n, ncols, ld, ldb,
               seed, traj0, round, k, mode, Zp, ldp, base_slot);
  else
    MQO_LAUNCH(k_reset_apply<false>, dim3(blocks_for(cnt)), dim3(256), 0, s, st, keys, Zb, X, V, lo, n, ncols, ld,
               ldb, seed, traj0, round, k, mode, Zp, ldp, base_slot);
}

void launch_pool_update(bool maxcut, const int8_t *Z, int32_t ld, const int64_t *vtx_off, int32_t G, int64_t n_total,
                        int32_t B, int32_t K, const int64_t *value, unsigned long long *hash, int8_t *taken,
                        const int8_t *pz_old, const int64_t *pv_old, const unsigned long long *ph_old,
                        int8_t *pz_new, int64_t *pv_new, unsigned long long *ph_new, int32_t *src, hipStream_t s) {
  // hashes of the round's columns of every graph
  MQO_LAUNCH(k_fill_i64, dim3(blocks_for((int64_t)G * B)), dim3(256), 0, s, reinterpret_cast<int64_t *>(hash),
             (int64_t)G * B, (int64_t)0);
  MQO_LAUNCH(k_col_hash, dim3(blocks_for(((n_total + 255) >> 8) * B)), dim3(256), 0, s, Z, vtx_off, G, n_total, B,
             ld, hash);
  // one workgroup per graph: its selection
  MQO_LAUNCH(k_pool_select, dim3((unsigned)G), dim3(256), 0, s, pv_old, ph_old, value, hash, K, B, maxcut ? 0 : 1,
             taken, pv_new, ph_new, src);
  MQO_LAUNCH(k_pool_copy, dim3(blocks_for(n_total * K)), dim3(256), 0, s, pz_old, Z, src, pz_new, vtx_off, G,
             n_total, K, ld);
}

void launch_pool_bases(const int64_t *pv, int32_t K, int32_t G, int32_t ncols, uint64_t seed, uint64_t round,
                       int32_t *base, hipStream_t s) {
  MQO_LAUNCH(k_pool_bases, dim3(blocks_for((int64_t)G * ncols)), dim3(256), 0, s, pv, K, G, ncols, seed, round, base);
}

void launch_mask_empty(int64_t *value, const int64_t *pv, int64_t count, hipStream_t s) {
  MQO_LAUNCH(k_mask_empty, dim3(blocks_for(count)), dim3(256), 0, s, value, pv, count);
}

void launch_sum_f64(const double *in, int64_t count, double *out, hipStream_t s) {
  MQO_LAUNCH(k_sum_f64, dim3(1), dim3(256), 0, s, in, count, out);
}

void launch_offer(const int8_t *Z, int32_t ld, const int64_t *cand, const int64_t *filled, int32_t K, int32_t G,
                  bool need_sol, const int64_t *voff, int64_t n_total, int64_t *sol_v, int8_t *sol_z,
                  int32_t *choice, hipStream_t s) {
  MQO_LAUNCH(k_offer_pick, dim3(blocks_for(G)), dim3(256), 0, s, cand, filled, K, G, (int32_t)need_sol, sol_v, choice);
  MQO_LAUNCH(k_offer_copy, dim3(blocks_for(n_total)), dim3(256), 0, s, Z, ld, choice, voff, G, sol_z, n_total);
}

void launch_strided_copy_i8(const int8_t *src, int32_t lds, int32_t cs, int8_t *dst, int32_t ldd, int32_t cd,
                            int64_t lo, int64_t n, hipStream_t s) {
  MQO_LAUNCH(k_strided_copy_i8, dim3(blocks_for(n)), dim3(256), 0, s, src, lds, cs, dst, ldd, cd, lo, n);
}

void launch_pick_best(const int64_t *best, int32_t G, int32_t B, int64_t *best_value, int32_t *best_b,
                      hipStream_t s) {
  MQO_LAUNCH(k_pick_best, dim3((unsigned)G), dim3(256), 0, s, best, G, B, best_value, best_b);
}

void launch_copy_best_x(const int8_t *Zb, int32_t B, const int64_t *voff, int32_t G, const int32_t *best_b,
                        int8_t *out, int64_t n_total, hipStream_t s) {
  MQO_LAUNCH(k_copy_best_x, dim3(blocks_for(n_total)), dim3(256), 0, s, Zb, B, voff, G, best_b, out, n_total);
}

void launch_gather_rowptr(const int32_t *row_ptr, const int64_t *voff, int32_t G, int32_t *out, hipStream_t s) {
  MQO_LAUNCH(k_gather_rowptr, dim3(blocks_for(G + 1)), dim3(256), 0, s, row_ptr, voff, G, out);
}

void launch_validate_rows(const int32_t *row_ptr, int64_t n, int64_t nnz, int32_t *err, hipStream_t s) {
  MQO_LAUNCH(k_validate_rows, dim3(blocks_for(n)), dim3(256), 0, s, row_ptr, n, nnz, err);
}

// hub list of one graph: each entry a row of [lo, lo + n) with degree >
// min_deg, strictly ascending (err |= 64 otherwise)
__global__ void k_validate_hubs(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ hubs, int64_t count,
                                int64_t lo, int64_t n, int32_t min_deg, int32_t *err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t r = hubs[i];
  if (r < lo || r >= lo + n || (i > 0 && hubs[i - 1] >= r) || row_ptr[r + 1] - row_ptr[r] <= min_deg)
    atomicOr(err, 64);
}

// number of rows of degree > min_deg
__global__ void k_count_hubs(const int32_t *__restrict__ row_ptr, int64_t n, int32_t min_deg, int32_t *count) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool hub = v < n && row_ptr[v + 1] - row_ptr[v] > min_deg;
  const unsigned long long b = __ballot(hub);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (int32_t)__popcll(b));
}

void launch_validate_hubs(const int32_t *row_ptr, const int32_t *hubs, int64_t count, int64_t lo, int64_t n,
                          int32_t min_deg, int32_t *err, hipStream_t s) {
  MQO_LAUNCH(k_validate_hubs, dim3(blocks_for(count)), dim3(256), 0, s, row_ptr, hubs, count, lo, n, min_deg, err);
}

void launch_count_hubs(const int32_t *row_ptr, int64_t n, int32_t min_deg, int32_t *count, hipStream_t s) {
  MQO_LAUNCH(k_count_hubs, dim3(blocks_for(n)), dim3(256), 0, s, row_ptr, n, min_deg, count);
}

void launch_validate_cols(const int32_t *row_ptr, const int32_t *col_idx, const int32_t *weight, const int64_t *voff,
                          int32_t G, int64_t n, int64_t nnz, int32_t *err, hipStream_t s) {
  MQO_LAUNCH(k_validate_cols, dim3(blocks_for(n)), dim3(256), 0, s, row_ptr, col_idx, weight, voff, G, n, nnz, err);
}

int64_t grid_blocks_x(int64_t nrows, StepCfg cfg) { return grid_rows(nrows, 1, cfg.lanes_log2, 1, 256).x; }

int64_t spmm_row_blocks(const GraphView &g, StepCfg cfg) {
  const int rows = spmm_rows(g, cfg.lanes_log2);
  return grid_rows((g.n + rows - 1) / rows, 1, cfg.lanes_log2, 1, 256).x;
}

template <int VEC>
struct ObjLaunch {
  template <int OBJ, bool W>
  static void run(const GraphView &g, const float *X, const float *scale, float *grad, double *part, int32_t ncols,
                  int32_t ld, int ll, float param, hipStream_t s) {
    const size_t lds = std::max(g.nhub ? hub_lds(W) : 0, part ? PARTIAL_LDS(VEC) : 0);
    const dim3 grid = spmm_grid(g, ncols, ll, VEC);
    if (spmm_rows(g, ll) == 2) {
      MQO_LAUNCH((k_objective_grad<VEC, OBJ, W, 2>), grid, dim3(256), lds, s, g, X, scale, grad, part, ncols, ld, ll,
                 param);
      return;
    }
    if (g.nhub > 0)  // uneven degrees: eight gathers in flight per lane group
      MQO_LAUNCH((k_objective_grad<VEC, OBJ, W, 1, 8>), grid, dim3(256), lds, s, g, X, scale, grad, part, ncols, ld,
                 ll, param);
    else
      MQO_LAUNCH((k_objective_grad<VEC, OBJ, W, 1>), grid, dim3(256), lds, s, g, X, scale, grad, part, ncols, ld, ll,
                 param);
  }
};

void launch_objective_grad(int form, const GraphView &g, const float *X, const float *scale, float *grad,
                           double *part, int32_t ncols, int32_t ld, StepCfg cfg, float param, hipStream_t s) {
  const bool w = g.weight != nullptr;
  const int ll = cfg.lanes_log2;
  if (cfg.vec == 4)
    dispatch_form<ObjLaunch<4>>(form, w, g, X, scale, grad, part, ncols, ld, ll, param, s);
  else if (cfg.vec == 2)
    dispatch_form<ObjLaunch<2>>(form, w, g, X, scale, grad, part, ncols, ld, ll, param, s);
  else
    dispatch_form<ObjLaunch<1>>(form, w, g, X, scale, grad, part, ncols, ld, ll, param, s);
}

void launch_reduce_partials(double *part, int64_t nblk, int32_t ncols, double *out, bool accumulate, hipStream_t s) {
  int32_t wlog2 = 0;
  while ((1 << wlog2) < ncols && wlog2 < 6) ++wlog2;
  const unsigned cx = (unsigned)((ncols + (1 << wlog2) - 1) >> wlog2);
  // at most two launches: one workgroup per column chunk sums up to F = 8 R
  // rows (8 loads per thread), so more than F partial rows first go through
  // one level of at most F slices of at least F rows each, written after
  // the partials (reduce_rows() leaves room for nblk / F + 1 of them)
  const int64_t F = 8 * (int64_t)(256 >> wlog2);
  const double *src = part;
  int64_t rows = nblk;
  if (rows > F) {
    const int64_t p = std::max(F, (rows + F - 1) / F);
    const int64_t slices = (rows + p - 1) / p;
    double *next = part + nblk * ncols;
    MQO_LAUNCH(k_reduce_partials, dim3(cx, (unsigned)slices), dim3(256), 0, s, src, rows, ncols, wlog2, p, next, 0);
    src = next;
    rows = slices;
  }
  MQO_LAUNCH(k_reduce_partials, dim3(cx, 1), dim3(256), 0, s, src, rows, ncols, wlog2, rows, out, (int32_t)accumulate);
}

template <int VEC>
struct AdjLaunch {
  template <int OBJ, bool W>
  static void run(const GraphView &g, const float *Xk, const float *lam_next, float *mu, float *lam, double *part,
                  int32_t ncols, int32_t ld, int ll, float alpha, float param, hipStream_t s) {
    const dim3 grid = spmm_grid(g, ncols, ll, VEC);
    const size_t lds_mu = std::max(g.nhub ? hub_lds(W) : 0, PARTIAL_LDS(VEC)), lds_lam = g.nhub ? hub_lds(W) : 0;
    if (spmm_rows(g, ll) == 2) {
      MQO_LAUNCH((k_adj_mu<VEC, OBJ, W, 2>), grid, dim3(256), lds_mu, s, g, Xk, lam_next, mu, part, ncols, ld, ll,
                 alpha, param);
      MQO_LAUNCH((k_adj_lambda<VEC, OBJ, W, 2>), grid, dim3(256), lds_lam, s, g, mu, lam, ncols, ld, ll, alpha, param);
      return;
    }
    if (g.nhub > 0) {  // uneven degrees: eight gathers in flight per lane group
      MQO_LAUNCH((k_adj_mu<VEC, OBJ, W, 1, 8>), grid, dim3(256), lds_mu, s, g, Xk, lam_next, mu, part, ncols, ld, ll,
                 alpha, param);
      MQO_LAUNCH((k_adj_lambda<VEC, OBJ, W, 1, 8>), grid, dim3(256), lds_lam, s, g, mu, lam, ncols, ld, ll, alpha,
                 param);
      return;
    }
    MQO_LAUNCH((k_adj_mu<VEC, OBJ, W, 1>), grid, dim3(256), lds_mu, s, g, Xk, lam_next, mu, part, ncols, ld, ll,
               alpha, param);
    MQO_LAUNCH((k_adj_lambda<VEC, OBJ, W, 1>), grid, dim3(256), lds_lam, s, g, mu, lam, ncols, ld, ll, alpha, param);
  }
};

void launch_adjoint_step(int form, const GraphView &g, const float *Xk, const float *lam_next, float *mu,
                         float *lam, double *part, int32_t ncols, int32_t ld, StepCfg cfg, float alpha, float param,
                         hipStream_t s) {
  const bool w = g.weight != nullptr;
  const int ll = cfg.lanes_log2;
  if (cfg.vec == 4)
    dispatch_form<AdjLaunch<4>>(form, w, g, Xk, lam_next, mu, lam, part, ncols, ld, ll, alpha, param, s);
  else if (cfg.vec == 2)
    dispatch_form<AdjLaunch<2>>(form, w, g, Xk, lam_next, mu, lam, part, ncols, ld, ll, alpha, param, s);
  else
    dispatch_form<AdjLaunch<1>>(form, w, g, Xk, lam_next, mu, lam, part, ncols, ld, ll, alpha, param, s);
}

}  // namespace mqo
