// Persistent tile plan.  One workgroup owns graph g and the trajectories
// b0 .. b0+T-1 of it; the iterate tile X[n_g][T] stays in LDS (double
// buffered: a step reads one buffer and writes the other, one barrier per
// step) for a whole round: reset (or x0) -> steps_per_round PGA steps ->
// threshold rounding -> neighbour counts -> 1-flip local search -> exact
// evaluation -> acceptance.  Only workgroup barriers are used; integer work
// arrays and the momentum live in a private global scratch region of the
// workgroup (L1/L2 resident).
//
// Step-loop shape (chosen by the autotuner): each lane owns VEC consecutive
// trajectories of one row (LDS reads of 4*VEC bytes); with CSR_LDS the
// graph's column indices are staged in LDS as 16-bit local ids so that a
// step touches no global memory at all.  With SB (single buffer) the tile
// is held once: a step gathers into registers (at most SB_ITEMS lane items
// per thread), then, after a barrier, writes the new iterate in place, so
// that twice the trajectories fit in LDS -- wider rows of the tile, whose
// random gathers then meet fewer LDS bank conflicts.
//
// Arithmetic per element is identical to the grid kernels (same operation
// order), so every plan gives bit-identical trajectories.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace mqo {

constexpr int TILE_MAX_T = 64;
constexpr int SB_ITEMS = 8;  // lane items per thread of a single-buffered step

template <int VEC>
__device__ __forceinline__ void lds_load(const float *p, float (&o)[VEC]) {
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

// LDS byte addresses as plain 32-bit integers: a neighbour's address is then
// one shift-and-add of its column id onto a per-lane base (the base folds in
// the buffer, the lane's trajectory offset and minus the graph's first
// vertex; the sum wraps modulo 2^32 to the exact in-range address).
typedef __attribute__((address_space(3))) const float lds_cfloat;

__device__ __forceinline__ uint32_t lds_byte_addr(const float *p) {
  return (uint32_t)(uintptr_t)(lds_cfloat *)p;
}

typedef float lds_f2 __attribute__((ext_vector_type(2)));
typedef float lds_f4 __attribute__((ext_vector_type(4)));

template <int VEC>
__device__ __forceinline__ void lds_load_addr(uint32_t byte_addr, float (&o)[VEC]) {
  if constexpr (VEC == 1) {
    o[0] = *(lds_cfloat *)(uintptr_t)byte_addr;
  } else if constexpr (VEC == 2) {
    const lds_f2 t = *(__attribute__((address_space(3))) const lds_f2 *)(uintptr_t)byte_addr;
    o[0] = t.x;
    o[1] = t.y;
  } else {
    const lds_f4 t = *(__attribute__((address_space(3))) const lds_f4 *)(uintptr_t)byte_addr;
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
  }
}

template <int VEC>
__device__ __forceinline__ void lds_store(float *p, const float (&o)[VEC]) {
  if constexpr (VEC == 1) {
    *p = o[0];
  } else if constexpr (VEC == 2) {
    *reinterpret_cast<float2 *>(p) = make_float2(o[0], o[1]);
  } else {
    *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
  }
}

// Dynamic LDS, in order: the iterate buffer(s), the graph's row_ptr, (with
// row order) the rows by descending degree as uint16, (CSR_LDS) the local
// column ids, (register shapes) the discrete state.  Byte offsets of the
// row order, the column ids and the state:
__host__ __device__ inline size_t tile_rord_offset(int64_t n_max, int T, bool single_buf) {
  const int64_t rowsX = (n_max > 256 ? n_max : 256) + 1;
  const size_t b =
      (size_t)((single_buf ? 1 : 2) * rowsX) * T * sizeof(float) + (size_t)(n_max + 1) * sizeof(int32_t);
  return (b + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t tile_cls_offset(int64_t n_max, int T, bool single_buf, bool row_order) {
  const size_t b = tile_rord_offset(n_max, T, single_buf) + (row_order ? (size_t)(n_max + 1) * sizeof(uint16_t) : 0);
  return (b + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t tile_state_offset(int64_t n_max, int T, int64_t nnz_max, bool csr_lds,
                                                    bool single_buf, bool row_order) {
  size_t b = tile_cls_offset(n_max, T, single_buf, row_order);
  if (csr_lds) b += (size_t)(nnz_max + 8) * sizeof(uint16_t);
  return (b + 15) & ~(size_t)15;
}

template <bool MAXCUT, bool WEIGHTED, int VEC, bool CSR_LDS, int DREG, int IPT, bool SB>
// Four register rows per lane need more than the 128 VGPRs a 1024-thread
// workgroup leaves, so that variant is built for at most 512 threads.
__global__ __launch_bounds__(IPT >= 4 ? 512 : 1024) void k_tile_round(TileArgs a) {
  extern __shared__ __align__(16) float smem[];
  __shared__ uint32_t s_prefix[TILE_MAX_T], s_krem[TILE_MAX_T], s_cnteq[TILE_MAX_T], s_tie[TILE_MAX_T];
  __shared__ int32_t s_sel_done[TILE_MAX_T], s_sel_left;
  __shared__ unsigned long long s_acc[2][TILE_MAX_T];
  __shared__ int32_t s_take[TILE_MAX_T];
  __shared__ int32_t s_active[2];
  // early exit: column still stepping in this round, its rounded point
  // failed the fixed-point test, PGA steps it executed (all rounds)
  __shared__ int32_t s_act[TILE_MAX_T], s_viol[TILE_MAX_T];
  __shared__ long long s_cnt[TILE_MAX_T];

  const int nthr = blockDim.x, tid = threadIdx.x;
  const int wave = tid >> 6, nwaves = nthr >> 6;
  // XCD-aware placement: the dispatch slots of one XCD (blockIdx % 8) take
  // consecutive (graph, tile) pairs, so a graph's CSR stays in one L2.
  const int32_t nwg = a.G * a.tiles;
  int32_t wid = blockIdx.x;
  if ((nwg & 7) == 0) wid = (int32_t)(blockIdx.x & 7) * (nwg >> 3) + (int32_t)(blockIdx.x >> 3);
  const int32_t g = a.gorder ? a.gorder[wid / a.tiles] : wid / a.tiles, tile = wid % a.tiles;
  const int64_t lo = a.vtx_off[g];
  const int32_t n = (int32_t)(a.vtx_off[g + 1] - lo);
  const int32_t T = a.T, lt = a.log2T;
  const int32_t b0 = tile * T;
  const int32_t cols = min(T, a.B - b0);
  const int32_t nT = n << lt;
  const int64_t traj0 = (int64_t)g * a.B + b0;
  const int64_t ldz = a.B;
  const int32_t ilo = (int32_t)lo;
  const bool momentum = a.mu != 0.0f;

  // both iterate buffers have rowsX rows; the last row stays 0 (padding
  // target of the register adjacency), rows 0..255 of xa also hold the reset
  // histogram
  const int32_t rowsX = max(a.n_max, 256) + 1;
  const int32_t zrow = rowsX - 1;
  float *xa = smem;                                                     // [rowsX][T]
  float *xb = SB ? smem : smem + (size_t)rowsX * T;                     // [rowsX][T] (SB: the same buffer)
  int32_t *rps = reinterpret_cast<int32_t *>(xb + (size_t)rowsX * T);  // [n_max+1] row_ptr of the graph
  // [n_max + 1] rows by descending degree (the general step loop's lane
  // items walk rows in this order)
  constexpr bool ROWORD = DREG == 0;
  uint16_t *rord = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(smem) + tile_rord_offset(a.n_max, T, SB));
  // [nnz_max + 8] local columns (CSR_LDS), 16-byte aligned for 8-wide reads
  uint16_t *cls =
      reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(smem) + tile_cls_offset(a.n_max, T, SB, ROWORD));
  // discrete state per (row, trajectory): in LDS after the CSR for the
  // register-adjacency shapes (small tiles), else in the workgroup's region
  // of the global scratch (L2-resident)
  const int64_t sbase = (int64_t)wid * a.n_max * T;
  const int64_t nTmax = (int64_t)a.n_max * T;
  char *sl = reinterpret_cast<char *>(smem) + tile_state_offset(a.n_max, T, a.nnz_max, CSR_LDS, SB, ROWORD);
  constexpr bool SLDS = DREG > 0;
  int8_t *zs = SLDS ? reinterpret_cast<int8_t *>(sl + 8 * nTmax) : a.zs + sbase;
  int32_t *nb = SLDS ? reinterpret_cast<int32_t *>(sl + 4 * nTmax) : a.nb + sbase;
  uint32_t *prio = SLDS ? reinterpret_cast<uint32_t *>(sl) : a.prio + sbase;  // also the reset keys
  int8_t *fl = SLDS ? reinterpret_cast<int8_t *>(sl + 9 * nTmax) : a.fl + sbase;
  float *vm = a.vm + sbase;
  const int32_t *ci = a.col_idx;
  const int32_t *wt = a.weight;

  if (tid < TILE_MAX_T) s_cnt[tid] = 0;
  const bool chk = a.check_every > 0;
  const int32_t e0 = a.row_ptr[lo];
  for (int32_t v = tid; v <= n; v += nthr) rps[v] = a.row_ptr[lo + v] - e0;
  const int32_t nnz_g = a.row_ptr[lo + n] - e0;
  const int32_t *cig = ci + e0;  // the graph's columns, global ids
  const int32_t *wtg = WEIGHTED ? wt + e0 : nullptr;
  if (CSR_LDS)
    for (int32_t j = tid; j < nnz_g + 8; j += nthr) cls[j] = j < nnz_g ? (uint16_t)(cig[j] - ilo) : (uint16_t)0;
  const int32_t k = (int32_t)floor(a.rho * (double)n);
  const int32_t ls_cap = 4 * (n + nnz_g) + 64;
  int32_t ls_total = 0;
  for (int32_t c = tid; c < T; c += nthr) {
    xa[zrow * T + c] = 0.0f;
    xb[zrow * T + c] = 0.0f;
  }
  // register adjacency (DREG > 0, unweighted graphs of degree <= DREG): lane
  // item i = row v, trajectory c keeps the LDS offsets of its neighbours in
  // ascending CSR order, padded with the zero row; adding the padding zeros
  // at the end of the sum leaves every result bit-identical
  // The LDS addresses of the neighbours in both iterate buffers are kept, so
  // that a step issues its DREG reads without address arithmetic.
  constexpr int RI = DREG > 0 ? IPT : 1, RD = DREG > 0 ? DREG : 1;
  const float *pa[RI][RD];
  const float *pb[RI][RD];
  float xr[RI];  // the lane's own iterate entries, kept across steps
  if constexpr (DREG > 0) {
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int32_t L = tid + i * nthr;
      const int32_t v = L < nT ? L >> lt : 0, c = L & (T - 1);
      const int32_t beg = L < nT ? a.row_ptr[lo + v] - e0 : 0, end = L < nT ? a.row_ptr[lo + v + 1] - e0 : 0;
#pragma unroll
      for (int kk = 0; kk < DREG; ++kk) {
        const int32_t off = beg + kk < end ? ((cig[beg + kk] - ilo) << lt) | c : (zrow << lt) | c;
        pa[i][kk] = xa + off;
        pb[i][kk] = xb + off;
      }
    }
  }
  __syncthreads();

  if constexpr (ROWORD) {
    // rows by descending degree: a counting sort over 256 bins of the
    // degree shifted right until the largest fits (ties in any order: a
    // row's arithmetic does not depend on the lane that runs it); the tile
    // is not written yet, so its first 1 KB holds the bins
    uint32_t *bins = reinterpret_cast<uint32_t *>(xa);
    if (tid == 0) s_sel_left = 0;
    for (int32_t h = tid; h < 256; h += nthr) bins[h] = 0u;
    __syncthreads();
    for (int32_t v = tid; v < n; v += nthr) atomicMax(&s_sel_left, rps[v + 1] - rps[v]);
    __syncthreads();
    int32_t shift = 0;
    while ((s_sel_left >> shift) > 255) ++shift;
    auto bin_of = [&](int32_t v) { return 255 - ((rps[v + 1] - rps[v]) >> shift); };
    for (int32_t v = tid; v < n; v += nthr) atomicAdd(&bins[bin_of(v)], 1u);
    __syncthreads();
    if (wave == 0) {  // exclusive scan: four bins per lane, then across the wavefront
      const int lane = tid & 63;
      uint32_t c[4], tot = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = bins[lane * 4 + q];
        tot += c[q];
      }
      uint32_t incl = tot;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
      }
      uint32_t run = incl - tot;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        bins[lane * 4 + q] = run;
        run += c[q];
      }
    }
    __syncthreads();
    for (int32_t v = tid; v < n; v += nthr) rord[atomicAdd(&bins[bin_of(v)], 1u)] = (uint16_t)v;
    __syncthreads();
  }

  // lane item I = VEC trajectories (from c0) of row v, the row at slot
  // I * VEC >> lt of the row order; returns the offset of its entries
  auto item_pos = [&](int32_t I, int32_t &v, int32_t &c0) {
    const int32_t L0 = I * VEC;
    v = ROWORD ? (int32_t)rord[L0 >> lt] : L0 >> lt;
    c0 = L0 & (T - 1);
    return (v << lt) | c0;
  };

  // The neighbours of row v in the iterate tile at src, VEC columns from c0
  // on, in ascending CSR order: visit(j, xu) for CSR entry j with the
  // neighbour's VEC entries (shared by the step's sums and the neighbour
  // counts of the rounding)
  auto row_gather = [&](const float *src, int32_t v, int32_t c0, auto &&visit) {
    const int32_t beg = rps[v], end = rps[v + 1];
    // neighbour u's entries at LDS byte (u << (lt + 2)) + ab: ab holds the
    // buffer, the lane's column c0 and (global column ids) minus the
    // graph's first vertex
    const uint32_t sh = (uint32_t)lt + 2u;
    const uint32_t ab = lds_byte_addr(src) + 4u * (uint32_t)c0 - (CSR_LDS ? 0u : ((uint32_t)ilo << sh));
    auto add_nbr = [&](int32_t j, int32_t col) {
      float xu[VEC];
      lds_load_addr<VEC>(((uint32_t)col << sh) + ab, xu);
      visit(j, xu);
    };
    if constexpr (CSR_LDS) {
      // eight local ids per 16-byte LDS read, blocks aligned to 8: the
      // row's first and last blocks masked, full blocks between
      auto block = [&](int32_t j0, bool masked) {
        const uint4 q = *reinterpret_cast<const uint4 *>(cls + j0);
        const uint32_t qw[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const int32_t j = j0 + kk;
          if (masked && (j < beg || j >= end)) continue;
          add_nbr(j, (int32_t)((qw[kk >> 1] >> (16 * (kk & 1))) & 0xffffu));
        }
      };
      int32_t j0 = beg & ~7;
      if (j0 < beg && j0 < end) {
        block(j0, true);
        j0 += 8;
      }
      for (; j0 + 8 <= end; j0 += 8) block(j0, false);
      if (j0 < end) block(j0, true);
    } else {
      // the first (end - beg) % 4 neighbours one by one, an odd group of
      // four, then pairs of groups whose column ids are loaded one group
      // ahead into two register sets in turn (past the row's end the
      // current pair's first group is loaded again, in bounds, and not used)
      int32_t j = beg;
      for (const int32_t j1 = beg + ((end - beg) & 3); j < j1; ++j) add_nbr(j, cig[j]);
      if ((end - j) & 4) {
        int32_t q[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) q[t] = cig[j + t];
#pragma unroll
        for (int t = 0; t < 4; ++t) add_nbr(j + t, q[t]);
        j += 4;
      }
      if (j < end) {
        int32_t qa[4], qb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) qa[t] = cig[j + t];
        while (true) {
#pragma unroll
          for (int t = 0; t < 4; ++t) qb[t] = cig[j + 4 + t];
#pragma unroll
          for (int t = 0; t < 4; ++t) add_nbr(j + t, qa[t]);
          const int32_t ja = j + 8 < end ? j + 8 : j;
#pragma unroll
          for (int t = 0; t < 4; ++t) qa[t] = cig[ja + t];
#pragma unroll
          for (int t = 0; t < 4; ++t) add_nbr(j + 4 + t, qb[t]);
          j += 8;
          if (j >= end) break;
        }
      }
    }
  };

  for (int32_t r = a.r0; r < a.r1; ++r) {
    // ------------------------------------------------------------ start point
    // round 0, or a fresh start of the outer loop (the host launches each
    // pass separately, its start written into x0)
    if (r == 0 || (a.restart_every > 0 && r % a.restart_every == 0)) {
      for (int32_t L = tid; L < nT; L += nthr) {
        const int32_t v = L >> lt, c = L & (T - 1);
        xa[L] = c < cols ? a.x0[(lo + v) * ldz + b0 + c] : 0.0f;
      }
    } else {
      if (k > 0) {
        // R = the k smallest (key, v) per column: 4 x 8-bit radix select
        for (int32_t L = tid; L < nT; L += nthr) {
          const int32_t v = L >> lt, c = L & (T - 1);
          prio[L] = c < cols ? philox_vertex(a.seed, PURPOSE_RESET, traj0 + c, r, v) : 0u;
        }
        uint32_t *hist = reinterpret_cast<uint32_t *>(xa);
        if (tid < T) {
          s_prefix[tid] = 0u;
          s_krem[tid] = (uint32_t)k;
          s_tie[tid] = (uint32_t)n;
          s_cnteq[tid] = 0u;
          s_sel_done[tid] = 0;
        }
        if (tid == 0) s_sel_left = cols;
        for (int pass = 0; pass < 4; ++pass) {
          for (int32_t h = tid; h < T * 256; h += nthr) hist[h] = 0u;
          __syncthreads();
          const int hs = 32 - 8 * pass, ds = 24 - 8 * pass;
          for (int32_t L = tid; L < nT; L += nthr) {
            const int32_t c = L & (T - 1);
            if (c < cols && !s_sel_done[c]) {
              const uint32_t key = prio[L];
              if (pass == 0 || (key >> hs) == s_prefix[c]) atomicAdd(&hist[c * 256 + ((key >> ds) & 255u)], 1u);
            }
          }
          __syncthreads();
          for (int32_t c = wave; c < cols; c += nwaves) {  // one wavefront per column
            if (s_sel_done[c]) continue;
            uint32_t d, before, at;
            wave_select_digit(hist + c * 256, s_krem[c], d, before, at);
            if ((tid & 63) == 0) {
              uint32_t pre = (s_prefix[c] << 8) | d;
              const uint32_t krem = s_krem[c] - before;
              s_krem[c] = krem;
              s_cnteq[c] = at;
              if (at == krem && pass < 3) {
                // every key with this prefix is taken: the selection is the
                // keys up to the prefix's largest completion, all ties kept
                pre = (uint32_t)((((uint64_t)pre + 1) << (24 - 8 * pass)) - 1);
                s_sel_done[c] = 1;
                atomicSub(&s_sel_left, 1);
              }
              s_prefix[c] = pre;
            }
          }
          __syncthreads();
          if (s_sel_left == 0) break;  // uniform
        }
        // more vertices share the threshold key than remain to be taken:
        // the lowest indices are kept (rare; sequential scan per column)
        if (tid < cols && s_cnteq[tid] != s_krem[tid]) {
          uint32_t cnt = 0;
          for (int32_t v = 0; v < n; ++v) {
            if (prio[(v << lt) | tid] == s_prefix[tid]) {
              if (++cnt == s_krem[tid]) {
                s_tie[tid] = (uint32_t)v;
                break;
              }
            }
          }
        }
        __syncthreads();
      }
      for (int32_t L = tid; L < nT; L += nthr) {
        const int32_t v = L >> lt, c = L & (T - 1);
        float x = 0.0f;
        if (c < cols) {
          // the incumbent, or the pool slot the trajectory restarts from
          const int32_t bs = a.base_slot ? a.base_slot[traj0 + c] : -1;
          const float base =
              (float)(bs >= 0 ? a.zp[(lo + v) * a.ldp + bs] : a.zbest[(lo + v) * ldz + b0 + c]);
          x = base;
          if (k > 0) {
            const uint32_t kk = prio[L];
            const bool sel = kk < s_prefix[c] || (kk == s_prefix[c] && (uint32_t)v <= s_tie[c]);
            if (sel) x = a.reset_mode == 0 ? 0.0f : (MAXCUT ? -base : 1.0f - base);
          }
        }
        xa[L] = x;
      }
    }
    if (momentum)
      for (int32_t L = tid; L < nT; L += nthr) vm[L] = 0.0f;
    __syncthreads();

    // ------------------------------------------------------------ PGA steps
    const int32_t nI = nT / VEC;  // lane items: VEC consecutive trajectories of one row
    if constexpr (DREG > 0) {
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const int32_t L = tid + i * nthr;
        xr[i] = L < nT ? xa[L] : 0.0f;
      }
    }
    // Step st reads buffer (st & 1 ? xb : xa) and writes the other.  With
    // check_every = c > 0 the steps run in chunks of c; after every chunk but
    // the last, columns whose rounded point is a fixed point of the projected
    // step stop for the rest of the round (their entries are copied through).
    if (tid < T) {
      s_act[tid] = tid < cols ? 1 : 0;
      s_viol[tid] = 0;
    }
    __syncthreads();
    int32_t done = 0;
    while (done < a.steps) {
      const int32_t len = chk ? min(a.check_every, a.steps - done) : a.steps - done;
      if (T == 1 && !s_act[0]) break;  // uniform: the workgroup's only trajectory stopped
      __syncthreads();
      if (tid < cols && s_act[tid]) s_cnt[tid] += len;
      if constexpr (DREG > 0) {
        // all neighbour reads of the lane's rows are independent LDS loads,
        // unconditional (padding reads the zero row) so that they issue back
        // to back
        // CHK (compile-time): stopped columns are copied through
        auto reg_step = [&](auto chk_tag, const float *const(&p)[RI][RD], float *dst) {
          constexpr bool CHK = decltype(chk_tag)::value;
#pragma unroll
          for (int i = 0; i < IPT; ++i) {
            const int32_t L = tid + i * nthr;
            if (L < nT) {
              if (CHK && T > 1 && !s_act[L & (T - 1)]) {
                dst[L] = xr[i];
                continue;
              }
              float acc = 0.0f;
#pragma unroll
              for (int kk = 0; kk < DREG; ++kk) acc = acc + *p[i][kk];
              const float gr = grad_from_sum<MAXCUT>(acc, a.param);
              float d = gr;
              if (momentum) {
                const float t = a.mu * vm[L];
                d = t + gr;
                vm[L] = d;
              }
              const float s = a.alpha * d;
              const float y = xr[i] + s;
              xr[i] = clip_box<MAXCUT>(y);
              dst[L] = xr[i];
            }
          }
          __syncthreads();
        };
        if (!chk) {
          for (int32_t st = done; st < done + len; st += 2) {
            reg_step(std::false_type{}, pa, xb);
            if (st + 1 < done + len) reg_step(std::false_type{}, pb, xa);
          }
        } else {
          for (int32_t st = done; st < done + len; ++st) {
            if (st & 1)
              reg_step(std::true_type{}, pb, xa);
            else
              reg_step(std::true_type{}, pa, xb);
          }
        }
      }
      if constexpr (DREG == 0) {
        // CHK (compile-time): stopped columns are copied through
        // the new iterate of lane item I (VEC trajectories of one row) from src
        auto item_step = [&](auto chk_tag, const float *src, int32_t I, float (&x)[VEC]) {
          constexpr bool CHK = decltype(chk_tag)::value;
          int32_t v, c0;
          const int32_t L0 = item_pos(I, v, c0);
          float acc[VEC];
#pragma unroll
          for (int i = 0; i < VEC; ++i) acc[i] = 0.0f;
          row_gather(src, v, c0, [&](int32_t j, const float (&xu)[VEC]) {
            if (WEIGHTED) {
              const float w = (float)wtg[j];
#pragma unroll
              for (int i = 0; i < VEC; ++i) {
                const float p = w * xu[i];
                acc[i] = acc[i] + p;
              }
            } else {
#pragma unroll
              for (int i = 0; i < VEC; ++i) acc[i] = acc[i] + xu[i];
            }
          });
          lds_load<VEC>(src + L0, x);
#pragma unroll
          for (int i = 0; i < VEC; ++i) {
            const float gr = grad_from_sum<MAXCUT>(acc[i], a.param);
            float d = gr;
            if (momentum) {
              const float t = a.mu * vm[L0 + i];
              d = t + gr;
              if (!CHK || s_act[c0 + i]) vm[L0 + i] = d;
            }
            const float sv = a.alpha * d;
            const float y = x[i] + sv;
            if (!CHK || s_act[c0 + i]) x[i] = clip_box<MAXCUT>(y);  // else copied through
          }
        };
        // CHK (compile-time): stopped columns are copied through
        auto gen_step = [&](auto chk_tag, int32_t st) {
          if constexpr (SB) {
            // every item of the thread into registers, then in place
            float xn[SB_ITEMS][VEC];
#pragma unroll
            for (int kq = 0; kq < SB_ITEMS; ++kq) {
              int32_t I = tid + kq * nthr;
              // opaque per step: keeps the items' row bounds and addresses
              // from being hoisted out of the step loop (they would hold
              // the registers the gathers need)
              __asm__ volatile("" : "+v"(I));
              if (I < nI) item_step(chk_tag, xa, I, xn[kq]);
            }
            __syncthreads();
#pragma unroll
            for (int kq = 0; kq < SB_ITEMS; ++kq) {
              const int32_t I = tid + kq * nthr;
              int32_t v, c0;
              if (I < nI) lds_store<VEC>(xa + item_pos(I, v, c0), xn[kq]);
            }
            __syncthreads();
          } else {
            const float *src = (st & 1) ? xb : xa;
            float *dst = (st & 1) ? xa : xb;
            for (int32_t I = tid; I < nI; I += nthr) {
              float x[VEC];
              item_step(chk_tag, src, I, x);
              int32_t v, c0;
              lds_store<VEC>(dst + item_pos(I, v, c0), x);
            }
            __syncthreads();
          }
        };
        for (int32_t st = done; st < done + len; ++st) {
          if (chk)
            gen_step(std::true_type{}, st);
          else
            gen_step(std::false_type{}, st);
        }
      }
      done += len;
      if (done < a.steps) {
        // the early-exit test on the current iterate
        const float *xc = (done & 1) ? xb : xa;
        // z_v rounded and sum the (weighted) count of its rounded neighbours;
        // the column fails when its rounded point moves under a step
        auto moves = [&](int32_t z, int32_t sum) {
          if (MAXCUT) {
            const int32_t st = z * sum;  // gradient -lambda - 2 t_v, 0 < lambda < 2
            return st > 0 || (st == 0 && z == 1);
          } else {
            return z ? sum != 0 : sum == 0;  // checker of Eq. (8), gamma > 1
          }
        };
        if constexpr (DREG == 0) {
          // per lane item, the neighbours rounded as read from the tile in
          // LDS (the gather loop of the steps)
          for (int32_t I = tid; I < nT / VEC; I += nthr) {
            int32_t v, c0;
            const int32_t L0 = item_pos(I, v, c0);
            bool any = false;
#pragma unroll
            for (int i = 0; i < VEC; ++i) any |= c0 + i < cols && s_act[c0 + i];
            if (!any) continue;
            int32_t cnt[VEC];
#pragma unroll
            for (int i = 0; i < VEC; ++i) cnt[i] = 0;
            row_gather(xc, v, c0, [&](int32_t j, const float (&xu)[VEC]) {
#pragma unroll
              for (int i = 0; i < VEC; ++i) {
                const int32_t zu = round_x<MAXCUT>(xu[i]);
                cnt[i] += WEIGHTED ? wtg[j] * zu : zu;
              }
            });
            float x[VEC];
            lds_load<VEC>(xc + L0, x);
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
              const int32_t c = c0 + i;
              if (c < cols && s_act[c] && moves(round_x<MAXCUT>(x[i]), cnt[i])) s_viol[c] = 1;
            }
          }
        } else {
          for (int32_t L = tid; L < nT; L += nthr) zs[L] = round_x<MAXCUT>(xc[L]);
          __syncthreads();
          for (int32_t L = tid; L < nT; L += nthr) {
            const int32_t v = L >> lt, c = L & (T - 1);
            if (c >= cols || !s_act[c]) continue;
            int32_t sum = 0;
            for (int32_t j = rps[v]; j < rps[v + 1]; ++j) {
              const int32_t u = CSR_LDS ? (int32_t)cls[j] : cig[j] - ilo;
              const int32_t zu = zs[(u << lt) | c];
              sum += WEIGHTED ? wtg[j] * zu : zu;
            }
            if (moves(zs[L], sum)) s_viol[c] = 1;
          }
        }
        __syncthreads();
        if (tid < T) {
          if (!s_viol[tid]) s_act[tid] = 0;
          s_viol[tid] = 0;
        }
        __syncthreads();
      }
    }
    const float *xf = (done & 1) ? xb : xa;

    // ------------------------------------------- rounding and neighbour counts
    if constexpr (DREG == 0) {
      // one pass over the lane items: the item's own entries rounded, its
      // neighbour counts taken from the rounded neighbours read straight
      // from the iterate tile in LDS (rounding a neighbour's entry again
      // gives the same integer the state holds)
      for (int32_t I = tid; I < nT / VEC; I += nthr) {
        int32_t v, c0;
        const int32_t L0 = item_pos(I, v, c0);
        int32_t cnt[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i) cnt[i] = 0;
        row_gather(xf, v, c0, [&](int32_t j, const float (&xu)[VEC]) {
#pragma unroll
          for (int i = 0; i < VEC; ++i) {
            const int32_t zu = round_x<MAXCUT>(xu[i]);
            cnt[i] += WEIGHTED ? wtg[j] * zu : zu;
          }
        });
        float x[VEC];
        lds_load<VEC>(xf + L0, x);
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
          zs[L0 + i] = (int8_t)round_x<MAXCUT>(x[i]);
          nb[L0 + i] = cnt[i];
        }
      }
      __syncthreads();
    } else {
      for (int32_t L = tid; L < nT; L += nthr) zs[L] = round_x<MAXCUT>(xf[L]);
      __syncthreads();
    }
    // With the degree-3 register adjacency the lane's neighbour items come
    // from its offset registers (item index = offset into xa; the padding
    // points past the last item) instead of the CSR in global memory (wider
    // shapes keep the CSR loops: the extra live registers would spill).
    constexpr bool REG_NBRS = DREG == 3;
    if constexpr (REG_NBRS) {
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const int32_t L = tid + i * nthr;
        if (L < nT) {
          int32_t s = 0;
#pragma unroll
          for (int kk = 0; kk < DREG; ++kk) {
            const int32_t Lu = (int32_t)(pa[i][kk] - xa);
            if (Lu < nT) s += zs[Lu];
          }
          nb[L] = s;
        }
      }
    } else if constexpr (DREG > 0) {
      for (int32_t L = tid; L < nT; L += nthr) {
        const int32_t v = L >> lt, c = L & (T - 1);
        int32_t s = 0;
        for (int32_t j = rps[v]; j < rps[v + 1]; ++j) {
          const int32_t u = CSR_LDS ? (int32_t)cls[j] : cig[j] - ilo;
          const int32_t zu = zs[(u << lt) | c];
          s += WEIGHTED ? wtg[j] * zu : zu;
        }
        nb[L] = s;
      }
    }

    // ------------------------------------------------------- local search
    if (a.ls) {
      for (int32_t L = tid; L < nT; L += nthr) {
        const int32_t v = L >> lt, c = L & (T - 1);
        prio[L] = philox_vertex(a.seed, PURPOSE_LS, traj0 + c, r, v);
      }
      if (tid == 0) s_active[0] = 0;
      __syncthreads();
      int32_t it = 0;
      while (true) {
        if constexpr (REG_NBRS) {
#pragma unroll
          for (int i = 0; i < IPT; ++i) {
            const int32_t L = tid + i * nthr;
            if (L < nT) {
              const int32_t v = L >> lt, c = L & (T - 1);
              int8_t f = 0;
              int32_t k1;
              if (c < cols && ls_candidate_t<MAXCUT>(zs[L], nb[L], k1)) {
                s_active[it & 1] = 1;
                const uint32_t pv = prio[L];
                f = 1;
#pragma unroll
                for (int kk = 0; kk < DREG; ++kk) {
                  const int32_t Lu = (int32_t)(pa[i][kk] - xa);
                  int32_t k1u;
                  if (Lu < nT && ls_candidate_t<MAXCUT>(zs[Lu], nb[Lu], k1u) &&
                      key_beats(k1u, prio[Lu], Lu >> lt, k1, pv, v))
                    f = 0;
                }
              }
              fl[L] = f;
            }
          }
        } else {
          for (int32_t L = tid; L < nT; L += nthr) {
            const int32_t v = L >> lt, c = L & (T - 1);
            int8_t f = 0;
            int32_t k1;
            if (c < cols && ls_candidate_t<MAXCUT>(zs[L], nb[L], k1)) {
              s_active[it & 1] = 1;
              const uint32_t pv = prio[L];
              f = 1;
              for (int32_t j = rps[v]; j < rps[v + 1]; ++j) {
                const int32_t u = CSR_LDS ? (int32_t)cls[j] : cig[j] - ilo;
                const int32_t Lu = (u << lt) | c;
                int32_t k1u;
                if (ls_candidate_t<MAXCUT>(zs[Lu], nb[Lu], k1u) && key_beats(k1u, prio[Lu], u, k1, pv, v)) {
                  f = 0;
                  break;
                }
              }
            }
            fl[L] = f;
          }
        }
        __syncthreads();
        if (!s_active[it & 1]) break;
        if (it >= ls_cap) {
          if (tid == 0) atomicOr(a.err, 1);
          break;
        }
        if (tid == 0) s_active[(it + 1) & 1] = 0;
        if constexpr (REG_NBRS) {
#pragma unroll
          for (int i = 0; i < IPT; ++i) {
            const int32_t L = tid + i * nthr;
            if (L < nT && fl[L]) {
              const int32_t z = zs[L];
              const int32_t zn = MAXCUT ? -z : 1 - z;
              zs[L] = (int8_t)zn;
              const int32_t dz = zn - z;
#pragma unroll
              for (int kk = 0; kk < DREG; ++kk) {
                const int32_t Lu = (int32_t)(pa[i][kk] - xa);
                if (Lu < nT) atomicAdd(&nb[Lu], dz);
              }
            }
          }
        } else {
          for (int32_t L = tid; L < nT; L += nthr) {
            if (fl[L]) {
              const int32_t v = L >> lt, c = L & (T - 1);
              const int32_t z = zs[L];
              const int32_t zn = MAXCUT ? -z : 1 - z;
              zs[L] = (int8_t)zn;
              const int32_t dz = zn - z;
              for (int32_t j = rps[v]; j < rps[v + 1]; ++j) {
                const int32_t u = CSR_LDS ? (int32_t)cls[j] : cig[j] - ilo;
                atomicAdd(&nb[(u << lt) | c], WEIGHTED ? dz * wtg[j] : dz);
              }
            }
          }
        }
        __syncthreads();
        ++it;
      }
      ls_total += it;
    }

    // ------------------------------------------------ evaluation, acceptance
    // every item of a thread belongs to trajectory tid % T: sum them in
    // registers, reduce over the wavefront's lanes of that trajectory, then
    // one LDS add per (wavefront, trajectory)
    if (tid < 2 * TILE_MAX_T) s_acc[tid / TILE_MAX_T][tid % TILE_MAX_T] = 0ull;
    __syncthreads();
    {
      long long a0 = 0, a1 = 0;
      for (int32_t L = tid; L < nT; L += nthr) {
        const int32_t v = L >> lt, c = L & (T - 1);
        if (c < cols) {
          const int32_t z = zs[L], s = nb[L];
          if (MAXCUT) {
            int32_t wsum = rps[v + 1] - rps[v];
            if (WEIGHTED) {
              wsum = 0;
              for (int32_t j = rps[v]; j < rps[v + 1]; ++j) wsum += wtg[j];
            }
            a0 += (long long)wsum - (long long)z * s;
          } else if (z) {
            a0 += 1;
            a1 += s;
          }
        }
      }
      const int width = T;  // T <= 64 divides the wavefront
      a0 = wave_sum_stride(a0, width);
      a1 = wave_sum_stride(a1, width);
      const int wl = tid & 63;
      if (wl < width) {
        if (a0) atomicAdd(&s_acc[0][wl], (unsigned long long)a0);
        if (!MAXCUT && a1) atomicAdd(&s_acc[1][wl], (unsigned long long)a1);
      }
    }
    __syncthreads();
    if (tid < cols) {
      int64_t value;
      if (MAXCUT)
        value = (long long)s_acc[0][tid] / 4;
      else
        value = s_acc[1][tid] == 0ull ? (int64_t)s_acc[0][tid] : -1;
      const int64_t t = traj0 + tid;
      const bool take = r == 0 || value > a.best[t];
      s_take[tid] = take ? 1 : 0;
      if (take) a.best[t] = value;
      if (a.vc) a.vc[t] = value;
    }
    __syncthreads();
    for (int32_t L = tid; L < nT; L += nthr) {
      const int32_t v = L >> lt, c = L & (T - 1);
      if (c < cols && s_take[c]) a.zbest[(lo + v) * ldz + b0 + c] = zs[L];
      if (c < cols && a.zc) a.zc[(lo + v) * ldz + b0 + c] = zs[L];
    }
    __syncthreads();
  }
  if (tid == 0) a.ls_iters[wid] = ls_total;
  if (tid < cols) a.steps_done[traj0 + tid] += s_cnt[tid];
}

bool tile_shape_ok(int64_t n_max, int T, int threads, int vec, bool csr_lds, int dreg, int ipt, bool sb) {
  if (!(T >= 1 && T <= TILE_MAX_T && (T & (T - 1)) == 0 && (threads == 256 || threads == 512 || threads == 1024) &&
        n_max >= 1 && n_max * T < (1LL << 30) && (vec == 1 || vec == 2 || vec == 4) && vec <= T &&
        (!csr_lds || n_max <= 65536) && (dreg > 0 || n_max <= 65536)))  // uint16 local ids / row order
    return false;
  // single buffer: every lane item of a step held in registers at once
  if (sb) return dreg == 0 && n_max * T <= (int64_t)SB_ITEMS * vec * threads;
  if (dreg == 0) return true;
  // register adjacency: one trajectory per lane item, at most ipt items per
  // lane; the shapes below fit the 128-VGPR budget of 1024-thread workgroups
  // without spilling
  const bool fits_regs = (dreg == 3 && ipt <= 2) || (dreg == 4 && ipt <= 2) || (dreg == 8 && ipt <= 2) ||
                         (dreg == 16 && ipt == 1) ||
                         (dreg <= 8 && ipt == 4 && threads <= 512);
  return fits_regs && (ipt == 1 || ipt == 2 || ipt == 4) && vec == 1 && !csr_lds &&
         n_max * T <= (int64_t)ipt * threads;
}

size_t tile_lds_bytes(int64_t n_max, int T, int64_t nnz_max, bool csr_lds, bool state_lds, bool sb) {
  size_t b = tile_state_offset(n_max, T, nnz_max, csr_lds, sb, !state_lds);
  // prio, nb (4 bytes), z, flag (1 byte) per (row, trajectory)
  if (state_lds) b += (size_t)n_max * T * 10;
  return (b + 15) & ~(size_t)15;
}

template <bool MC, bool W, int VEC, bool CL, int DREG, int IPT, bool SB = false>
static hipError_t tile_launch_t(const TileArgs &a, int threads, hipStream_t s) {
  const size_t lds = tile_lds_bytes(a.n_max, a.T, a.nnz_max, CL, DREG > 0, SB);
  auto kern = k_tile_round<MC, W, VEC, CL, DREG, IPT, SB>;
  // the dynamic-LDS limit only ever grows; raise it when a launch needs more
  // (per device; callers hold the library's host lock)
  static int limit_set[64] = {0};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64 || (int)lds > limit_set[dev]) {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) limit_set[dev] = (int)lds;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)(a.G * a.tiles)), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <bool MC, int DREG>
static hipError_t tile_launch_reg(const TileArgs &a, int threads, hipStream_t s) {
  if (DREG == 16 || a.ipt == 1) return tile_launch_t<MC, false, 1, false, DREG, 1>(a, threads, s);
  if (a.ipt == 2) return tile_launch_t<MC, false, 1, false, DREG, DREG == 16 ? 1 : 2>(a, threads, s);
  return tile_launch_t<MC, false, 1, false, DREG, DREG == 16 ? 1 : 4>(a, threads, s);
}

template <bool MC, bool W>
static hipError_t tile_launch_mw(const TileArgs &a, int threads, hipStream_t s) {
  if (!W && a.dreg > 0) {
    switch (a.dreg) {
      case 3: return tile_launch_reg<MC, 3>(a, threads, s);
      case 4: return tile_launch_reg<MC, 4>(a, threads, s);
      case 8: return tile_launch_reg<MC, 8>(a, threads, s);
      default: return tile_launch_reg<MC, 16>(a, threads, s);
    }
  }
  if (a.sb) {
    if (a.csr_lds) {
      switch (a.vec) {
        case 4: return tile_launch_t<MC, W, 4, true, 0, 1, true>(a, threads, s);
        case 2: return tile_launch_t<MC, W, 2, true, 0, 1, true>(a, threads, s);
        default: return tile_launch_t<MC, W, 1, true, 0, 1, true>(a, threads, s);
      }
    }
    switch (a.vec) {
      case 4: return tile_launch_t<MC, W, 4, false, 0, 1, true>(a, threads, s);
      case 2: return tile_launch_t<MC, W, 2, false, 0, 1, true>(a, threads, s);
      default: return tile_launch_t<MC, W, 1, false, 0, 1, true>(a, threads, s);
    }
  }
  if (a.csr_lds) {
    switch (a.vec) {
      case 4: return tile_launch_t<MC, W, 4, true, 0, 1>(a, threads, s);
      case 2: return tile_launch_t<MC, W, 2, true, 0, 1>(a, threads, s);
      default: return tile_launch_t<MC, W, 1, true, 0, 1>(a, threads, s);
    }
  }
  switch (a.vec) {
    case 4: return tile_launch_t<MC, W, 4, false, 0, 1>(a, threads, s);
    case 2: return tile_launch_t<MC, W, 2, false, 0, 1>(a, threads, s);
    default: return tile_launch_t<MC, W, 1, false, 0, 1>(a, threads, s);
  }
}

hipError_t launch_tile_round(bool maxcut, bool weighted, const TileArgs &a, int threads, hipStream_t s) {
  if (!tile_shape_ok(a.n_max, a.T, threads, a.vec, a.csr_lds != 0, a.dreg, a.ipt, a.sb != 0))
    return hipErrorInvalidValue;
  if (weighted && a.dreg > 0) return hipErrorInvalidValue;
  if (maxcut) return weighted ? tile_launch_mw<true, true>(a, threads, s) : tile_launch_mw<true, false>(a, threads, s);
  return tile_launch_mw<false, false>(a, threads, s);
}

}  // namespace mqo
