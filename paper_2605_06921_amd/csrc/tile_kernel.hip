// Persistent tile plan.  One workgroup owns graph g and the trajectories
// b0 .. b0+T-1 of it; the iterate tile X[n_g][T] stays in LDS (double
// buffered: a step reads one buffer and writes the other, one barrier per
// step) for a whole round: reset (or x0) -> steps_per_round PGA steps ->
// threshold rounding -> neighbour counts -> 1-flip local search -> exact
// evaluation -> acceptance.  Only workgroup barriers are used; integer work
// arrays and the momentum live in a private global scratch region of the
// workgroup (L1/L2 resident).
//
// Arithmetic per element is identical to the grid kernels (same operation
// order), so every plan gives bit-identical trajectories.
#include "common.h"
#include "kernels.h"

namespace mqo {

constexpr int TILE_MAX_T = 64;

template <bool MAXCUT, bool WEIGHTED, bool MOMENTUM>
__global__ __launch_bounds__(1024) void k_tile_round(TileArgs a) {
  extern __shared__ float smem[];
  __shared__ uint32_t s_prefix[TILE_MAX_T], s_krem[TILE_MAX_T], s_cnteq[TILE_MAX_T], s_tie[TILE_MAX_T];
  __shared__ unsigned long long s_acc[2][TILE_MAX_T];
  __shared__ int32_t s_take[TILE_MAX_T];
  __shared__ int32_t s_active[2];

  const int nthr = blockDim.x, tid = threadIdx.x;
  // XCD-aware placement: the dispatch slots of one XCD (blockIdx % 8) take
  // consecutive (graph, tile) pairs, so a graph's CSR stays in one L2.
  const int32_t nwg = a.G * a.tiles;
  int32_t wid = blockIdx.x;
  if ((nwg & 7) == 0) wid = (int32_t)(blockIdx.x & 7) * (nwg >> 3) + (int32_t)(blockIdx.x >> 3);
  const int32_t g = wid / a.tiles, tile = wid % a.tiles;
  const int64_t lo = a.vtx_off[g];
  const int32_t n = (int32_t)(a.vtx_off[g + 1] - lo);
  const int32_t T = a.T, lt = a.log2T;
  const int32_t b0 = tile * T;
  const int32_t cols = min(T, a.B - b0);
  const int32_t nT = n << lt;
  const int64_t traj0 = (int64_t)g * a.B + b0;
  const int64_t ldz = a.B;
  const int32_t ilo = (int32_t)lo;

  const int32_t rowsA = max(a.n_max, 256);
  float *xa = smem;                                                       // [rowsA][T], also the reset histogram
  float *xb = smem + (size_t)rowsA * T;                                   // [n_max][T]
  int32_t *rps = reinterpret_cast<int32_t *>(xb + (size_t)a.n_max * T);  // [n+1] row_ptr of the graph
  const int64_t sbase = (int64_t)wid * a.n_max * T;
  int8_t *zs = a.zs + sbase;
  int32_t *nb = a.nb + sbase;
  uint32_t *prio = a.prio + sbase;  // also the reset keys
  int8_t *fl = a.fl + sbase;
  float *vm = MOMENTUM ? a.vm + sbase : nullptr;
  const int32_t *ci = a.col_idx;
  const int32_t *wt = a.weight;

  for (int32_t v = tid; v <= n; v += nthr) rps[v] = a.row_ptr[lo + v];
  const int32_t nnz_g = a.row_ptr[lo + n] - a.row_ptr[lo];
  const int32_t k = (int32_t)floor(a.rho * (double)n);
  const int32_t ls_cap = 4 * (n + nnz_g) + 64;
  int32_t ls_total = 0;
  __syncthreads();

  for (int32_t r = a.r0; r < a.r1; ++r) {
    // ------------------------------------------------------------ start point
    if (r == 0) {
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
        }
        for (int pass = 0; pass < 4; ++pass) {
          for (int32_t h = tid; h < T * 256; h += nthr) hist[h] = 0u;
          __syncthreads();
          const int hs = 32 - 8 * pass, ds = 24 - 8 * pass;
          for (int32_t L = tid; L < nT; L += nthr) {
            const int32_t c = L & (T - 1);
            if (c < cols) {
              const uint32_t key = prio[L];
              if (pass == 0 || (key >> hs) == s_prefix[c]) atomicAdd(&hist[c * 256 + ((key >> ds) & 255u)], 1u);
            }
          }
          __syncthreads();
          if (tid < cols) {
            uint32_t cum = 0, d = 0, hv = 0;
            const uint32_t kr = s_krem[tid];
            for (d = 0; d < 256; ++d) {
              hv = hist[tid * 256 + d];
              if (cum + hv >= kr) break;
              cum += hv;
            }
            if (d > 255) d = 255;
            s_prefix[tid] = (s_prefix[tid] << 8) | d;
            s_krem[tid] = kr - cum;
            s_cnteq[tid] = hv;
          }
          __syncthreads();
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
          const float base = (float)a.zbest[(lo + v) * ldz + b0 + c];
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
    if (MOMENTUM)
      for (int32_t L = tid; L < nT; L += nthr) vm[L] = 0.0f;
    __syncthreads();

    // ------------------------------------------------------------ PGA steps
    for (int32_t st = 0; st < a.steps; ++st) {
      const float *src = (st & 1) ? xb : xa;
      float *dst = (st & 1) ? xa : xb;
      for (int32_t L = tid; L < nT; L += nthr) {
        const int32_t v = L >> lt, c = L & (T - 1);
        const int32_t beg = rps[v], end = rps[v + 1];
        float acc = 0.0f;
#pragma unroll 4
        for (int32_t j = beg; j < end; ++j) {
          const int32_t u = ci[j] - ilo;
          const float xu = src[(u << lt) | c];
          if (WEIGHTED) {
            const float p = (float)wt[j] * xu;
            acc = acc + p;
          } else {
            acc = acc + xu;
          }
        }
        const float gr = grad_from_sum<MAXCUT>(acc, a.param);
        float d = gr;
        if (MOMENTUM) {
          const float t = a.mu * vm[L];
          d = t + gr;
          vm[L] = d;
        }
        const float s = a.alpha * d;
        const float y = src[L] + s;
        dst[L] = clip_box<MAXCUT>(y);
      }
      __syncthreads();
    }
    const float *xf = (a.steps & 1) ? xb : xa;

    // ------------------------------------------- rounding and neighbour counts
    for (int32_t L = tid; L < nT; L += nthr) zs[L] = round_x<MAXCUT>(xf[L]);
    __syncthreads();
    for (int32_t L = tid; L < nT; L += nthr) {
      const int32_t v = L >> lt, c = L & (T - 1);
      int32_t s = 0;
      for (int32_t j = rps[v]; j < rps[v + 1]; ++j) {
        const int32_t u = ci[j] - ilo;
        const int32_t zu = zs[(u << lt) | c];
        s += WEIGHTED ? wt[j] * zu : zu;
      }
      nb[L] = s;
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
        for (int32_t L = tid; L < nT; L += nthr) {
          const int32_t v = L >> lt, c = L & (T - 1);
          int8_t f = 0;
          int32_t k1;
          if (c < cols && ls_candidate_t<MAXCUT>(zs[L], nb[L], k1)) {
            s_active[it & 1] = 1;
            const uint32_t pv = prio[L];
            f = 1;
            for (int32_t j = rps[v]; j < rps[v + 1]; ++j) {
              const int32_t u = ci[j] - ilo;
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
        __syncthreads();
        if (!s_active[it & 1]) break;
        if (it >= ls_cap) {
          if (tid == 0) atomicOr(a.err, 1);
          break;
        }
        if (tid == 0) s_active[(it + 1) & 1] = 0;
        for (int32_t L = tid; L < nT; L += nthr) {
          if (fl[L]) {
            const int32_t v = L >> lt, c = L & (T - 1);
            const int32_t z = zs[L];
            const int32_t zn = MAXCUT ? -z : 1 - z;
            zs[L] = (int8_t)zn;
            const int32_t dz = zn - z;
            for (int32_t j = rps[v]; j < rps[v + 1]; ++j) {
              const int32_t u = ci[j] - ilo;
              atomicAdd(&nb[(u << lt) | c], WEIGHTED ? dz * wt[j] : dz);
            }
          }
        }
        __syncthreads();
        ++it;
      }
      ls_total += it;
    }

    // ------------------------------------------------ evaluation, acceptance
    if (tid < 2 * TILE_MAX_T) s_acc[tid / TILE_MAX_T][tid % TILE_MAX_T] = 0ull;
    __syncthreads();
    for (int32_t L = tid; L < nT; L += nthr) {
      const int32_t v = L >> lt, c = L & (T - 1);
      if (c < cols) {
        const int32_t z = zs[L], s = nb[L];
        if (MAXCUT) {
          int32_t wsum = rps[v + 1] - rps[v];
          if (WEIGHTED) {
            wsum = 0;
            for (int32_t j = rps[v]; j < rps[v + 1]; ++j) wsum += wt[j];
          }
          const long long a0 = (long long)wsum - (long long)z * s;
          if (a0) atomicAdd(&s_acc[0][c], (unsigned long long)a0);
        } else if (z) {
          atomicAdd(&s_acc[0][c], 1ull);
          if (s) atomicAdd(&s_acc[1][c], (unsigned long long)s);
        }
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
    }
    __syncthreads();
    for (int32_t L = tid; L < nT; L += nthr) {
      const int32_t v = L >> lt, c = L & (T - 1);
      if (c < cols && s_take[c]) a.zbest[(lo + v) * ldz + b0 + c] = zs[L];
    }
    __syncthreads();
  }
  if (tid == 0) a.ls_iters[wid] = ls_total;
}

bool tile_shape_ok(int64_t n_max, int T, int threads) {
  return T >= 1 && T <= TILE_MAX_T && (T & (T - 1)) == 0 && (threads == 256 || threads == 512 || threads == 1024) &&
         n_max >= 1 && n_max * T < (1LL << 30);
}

size_t tile_lds_bytes(int64_t n_max, int T) {
  const int64_t rowsA = n_max > 256 ? n_max : 256;
  return (size_t)(rowsA + n_max) * T * sizeof(float) + (size_t)(n_max + 1) * sizeof(int32_t);
}

template <bool MC, bool W, bool M>
static hipError_t tile_launch_t(const TileArgs &a, int threads, hipStream_t s) {
  const size_t lds = tile_lds_bytes(a.n_max, a.T);
  auto kern = k_tile_round<MC, W, M>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3((unsigned)(a.G * a.tiles)), dim3(threads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_tile_round(bool maxcut, bool weighted, bool momentum, const TileArgs &a, int threads,
                             hipStream_t s) {
  if (!tile_shape_ok(a.n_max, a.T, threads)) return hipErrorInvalidValue;
  if (maxcut) {
    if (weighted)
      return momentum ? tile_launch_t<true, true, true>(a, threads, s) : tile_launch_t<true, true, false>(a, threads, s);
    return momentum ? tile_launch_t<true, false, true>(a, threads, s) : tile_launch_t<true, false, false>(a, threads, s);
  }
  return momentum ? tile_launch_t<false, false, true>(a, threads, s) : tile_launch_t<false, false, false>(a, threads, s);
}

}  // namespace mqo
