// Host-side launchers of the libmqo kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace mqo {

// Step-kernel shape: each lane owns `vec` consecutive columns, 2^lanes_log2
// lanes share one row.
struct StepCfg {
  int vec;
  int lanes_log2;
};

StepCfg default_step_cfg(int32_t ncols, int32_t ld);
int64_t grid_blocks_x(int64_t nrows, StepCfg cfg);
// row workgroups of a sparse-product launch over graph g (without hub workgroups)
int64_t spmm_row_blocks(const GraphView &g, StepCfg cfg);

// start: index of the fresh start (0 = the first; the outer loop's later
// starts use 1, 2, ...)
void launch_init_uniform(bool maxcut, float *X, int64_t lo, int64_t n, int32_t ncols, int32_t ld, uint64_t seed,
                         uint64_t traj0, hipStream_t s, uint64_t start = 0);
void launch_init_degree(bool maxcut, float *X, const int32_t *row_ptr, int32_t *dmax_scratch, int64_t lo, int64_t n,
                        int32_t ncols, int32_t ld, uint64_t seed, uint64_t traj0, float sigma, hipStream_t s,
                        uint64_t start = 0);
void launch_degree_max(const int32_t *row_ptr, int64_t n, int32_t *out, hipStream_t s);
// form: OBJ_H / OBJ_FB / OBJ_FL / OBJ_FP / OBJ_FA (common.h).
// colact: per-column active flags (0 = stopped for the round: copied
// through), or nullptr for all active
void launch_pga_step(int form, const GraphView &g, const float *X, float *Xn, float *V, int32_t ncols, int32_t ld,
                     StepCfg cfg, float alpha, float mu, float param, hipStream_t s, const int8_t *colact = nullptr);
void launch_active_update(int8_t *colact, const int8_t *fixed, int32_t ncols, hipStream_t s);
void launch_fill_i8(int8_t *p, int64_t count, int8_t v, hipStream_t s);
void launch_add_i64(int64_t *p, int64_t count, int64_t v, hipStream_t s);
// *out = sum_t steps[t] * nnz of t's graph (rpat: row_ptr at the G+1 graph boundaries)
void launch_edge_updates(const int64_t *steps, const int32_t *rpat, int32_t G, int32_t B, int64_t *out,
                         hipStream_t s);
void launch_count_steps(const int8_t *colact, int64_t *steps, int32_t ncols, int32_t len, hipStream_t s);
void launch_copy_f32(const float *a, float *b, int64_t count, hipStream_t s);
void launch_strided_copy_f32(const float *src, int32_t lds, int32_t cs, float *dst, int32_t ldd, int32_t cd,
                             int64_t lo, int64_t n, hipStream_t s);
void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s);
void launch_fill_i64(int64_t *p, int64_t count, int64_t v, hipStream_t s);
void launch_fill_f32(float *p, int64_t count, float v, hipStream_t s);
void launch_round(bool maxcut, const float *X, int8_t *Z, int64_t lo, int64_t n, int32_t ncols, int32_t ld,
                  hipStream_t s);
// acc: 3 * ncols int64 scratch
void launch_evaluate(bool maxcut, const GraphView &g, const int8_t *Z, int32_t *NB, long long *acc, int64_t *value,
                     int64_t *conflicts, int8_t *fixed, int32_t ncols, int32_t ld, hipStream_t s);
void launch_ls_prio(uint32_t *PRIO, int64_t lo, int64_t n, int32_t ncols, int32_t ld, uint64_t seed, uint64_t traj0,
                    uint64_t round, hipStream_t s);
void launch_ls_iteration(bool maxcut, const GraphView &g, int8_t *Z, int32_t *NB, const uint32_t *PRIO, int8_t *F,
                         int32_t *active, const int32_t *prev_active, int32_t ncols, int32_t ld, double mean_degree,
                         hipStream_t s);
// priorities of purpose SWAP for the pair moves
void launch_swap_prio(uint32_t *PRIO, int64_t lo, int64_t n, int32_t ncols, int32_t ld, uint64_t seed,
                      uint64_t traj0, uint64_t round, hipStream_t s);
// One parallel pair-move iteration ((1,2)-swap for MIS, 2-flip for MaxCut)
// on a 1-flip optimum, in two launches: the candidates (MIS proposals /
// best improving pair per vertex) into T0..T2 (int32 scratch [n][ld] each),
// then selection and application.  NB must hold A Z; *active is set when a
// move was applied (the caller clears it).
// TB: tightness bits, 8 * rows * ceil(ncols / 64) bytes, 8-byte aligned
void launch_pair_candidates(bool maxcut, const GraphView &g, const int8_t *Z, const int32_t *NB,
                            const uint32_t *PRIO, int32_t *T0, int32_t *T1, int32_t *T2, uint32_t *TB, int32_t ncols,
                            int32_t ld, double mean_degree, hipStream_t s);
void launch_pair_apply(bool maxcut, const GraphView &g, int8_t *Z, int32_t *NB, const uint32_t *PRIO, int8_t *F,
                       const int32_t *T0, const int32_t *T1, const int32_t *T2, int32_t *active, int32_t ncols,
                       int32_t ld, double mean_degree, hipStream_t s);
void launch_accept(const int8_t *Z, int8_t *Zb, const int64_t *value, int64_t *best, int64_t lo, int64_t n,
                   int32_t ncols, int32_t ld, int32_t ldb, bool first, hipStream_t s);
size_t reset_scratch_bytes(int32_t ncols);
// Zp / base_slot (optional): column c starts from pool slot base_slot[c] of
// Zp ([n][ldp]) instead of its incumbent when base_slot[c] >= 0
void launch_reset(bool maxcut, const int8_t *Zb, int32_t ldb, const uint32_t *keys, float *X, float *V, int64_t lo,
                  int64_t n, int32_t ncols, int32_t ld, uint64_t seed, uint64_t traj0, uint64_t round, int32_t k,
                  int32_t mode, void *scratch, hipStream_t s, const int8_t *Zp = nullptr, int32_t ldp = 0,
                  const int32_t *base_slot = nullptr);
// pmQO pool of every graph of the batch (vtx_off: device [G+1]): per graph,
// TopK of the old pool (pz_old [n_total][K], pv_old / ph_old [G][K]) united
// with the round's columns of Z (values value [G][B]) into pz_new / pv_new /
// ph_new.  hash: [G][B] scratch, taken: G (K + B) bytes, src: [G][K].
void launch_pool_update(bool maxcut, const int8_t *Z, int32_t ld, const int64_t *vtx_off, int32_t G, int64_t n_total,
                        int32_t B, int32_t K, const int64_t *value, unsigned long long *hash, int8_t *taken,
                        const int8_t *pz_old, const int64_t *pv_old, const unsigned long long *ph_old,
                        int8_t *pz_new, int64_t *pv_new, unsigned long long *ph_new, int32_t *src, hipStream_t s);
// base slot of every trajectory g ncols + c (pv [G][K]: the pool values)
void launch_pool_bases(const int64_t *pv, int32_t K, int32_t G, int32_t ncols, uint64_t seed, uint64_t round,
                       int32_t *base, hipStream_t s);
void launch_mask_empty(int64_t *value, const int64_t *pv, int64_t count, hipStream_t s);
// *out = sum of in[0 .. count) in a fixed order (one workgroup)
void launch_sum_f64(const double *in, int64_t count, double *out, hipStream_t s);
// best set of the pool modes: graph g is offered the K candidates
// cand[g K + c] (columns c of Z, leading dimension ld) in column order and
// takes each that is strictly above sol_v[g]; filled (optional): only
// columns with filled[g K + c] != INT64_MIN count; need_sol: graphs with no
// set yet (sol_v == INT64_MIN) take nothing.  choice: [G] scratch.
void launch_offer(const int8_t *Z, int32_t ld, const int64_t *cand, const int64_t *filled, int32_t K, int32_t G,
                  bool need_sol, const int64_t *voff, int64_t n_total, int64_t *sol_v, int8_t *sol_z,
                  int32_t *choice, hipStream_t s);
void launch_strided_copy_i8(const int8_t *src, int32_t lds, int32_t cs, int8_t *dst, int32_t ldd, int32_t cd,
                            int64_t lo, int64_t n, hipStream_t s);
void launch_pick_best(const int64_t *best, int32_t G, int32_t B, int64_t *best_value, int32_t *best_b, hipStream_t s);
void launch_copy_best_x(const int8_t *Zb, int32_t B, const int64_t *voff, int32_t G, const int32_t *best_b,
                        int8_t *out, int64_t n_total, hipStream_t s);
void launch_gather_rowptr(const int32_t *row_ptr, const int64_t *voff, int32_t G, int32_t *out, hipStream_t s);
void launch_validate_rows(const int32_t *row_ptr, int64_t n, int64_t nnz, int32_t *err, hipStream_t s);
void launch_validate_hubs(const int32_t *row_ptr, const int32_t *hubs, int64_t count, int64_t lo, int64_t n,
                          int32_t min_deg, int32_t *err, hipStream_t s);
void launch_count_hubs(const int32_t *row_ptr, int64_t n, int32_t min_deg, int32_t *count, hipStream_t s);
// safe to run in the same pass as the row check (skips rows with a bad range)
void launch_validate_cols(const int32_t *row_ptr, const int32_t *col_idx, const int32_t *weight, const int64_t *voff,
                          int32_t G, int64_t n, int64_t nnz, int32_t *err, hipStream_t s);
void launch_objective_grad(int form, const GraphView &g, const float *X, const float *scale, float *grad,
                           double *part, int32_t ncols, int32_t ld, StepCfg cfg, float param, hipStream_t s);
// partial rows [nblk][ncols] followed by room for reduce_rows(nblk) more
// rows (the reduction's intermediate levels)
inline int64_t reduce_rows(int64_t nblk) { return nblk / 7 + 64; }
void launch_reduce_partials(double *part, int64_t nblk, int32_t ncols, double *out, bool accumulate, hipStream_t s);
void launch_adjoint_step(int form, const GraphView &g, const float *Xk, const float *lam_next, float *mu,
                         float *lam, double *part, int32_t ncols, int32_t ld, StepCfg cfg, float alpha, float param,
                         hipStream_t s);

// address on the current device of the library's own MQO_STATIC_SCRATCH_BYTES
// of device scratch (looked up once per device)
hipError_t static_scratch_address(void **out);

// ---------------------------------------------------------------------------
// persistent tile plan: one workgroup owns (graph, T trajectories) with the
// iterate tile resident in LDS for a whole round
// ---------------------------------------------------------------------------
struct TileArgs {
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const int32_t *weight;
  const int64_t *vtx_off;  // device [G+1]
  // device [G]: the graph of each graph slot of the launch order (nullptr:
  // slot g is graph g)
  const int32_t *gorder;
  int32_t G, B, T, log2T, tiles;
  int32_t n_max;    // scratch stride (rows)
  int32_t nnz_max;  // largest graph's stored entries
  int32_t vec;      // trajectories per lane in the step loop (1, 2, 4)
  int32_t csr_lds;  // stage the graph's columns in LDS (16-bit local ids)
  int32_t dreg;     // > 0: neighbour offsets held in registers, padded to dreg
  int32_t ipt;      // lane items per thread in the register-adjacency path
  int32_t sb;       // 1: one iterate buffer, steps gather into registers first
  int32_t steps, r0, r1, reset_mode, ls;
  int32_t check_every;  // > 0: early-exit test after every check_every steps of a round
  int32_t restart_every;  // > 0: round r with r % restart_every == 0 starts from x0 (a fresh start)
  // the pmQO pool (launches of one round): the round's candidates out
  // (zc [n_total][B] with their values vc [G*B]), and the reset of round
  // r > 0 from pool slot base_slot[t] of zp ([n_total][ldp]) when >= 0
  int8_t *zc;
  int64_t *vc;
  const int8_t *zp;
  int32_t ldp;
  const int32_t *base_slot;
  float alpha, mu, param;
  double rho;
  uint64_t seed;
  const float *x0;  // [n_total][B], the start of round 0 and of every fresh start
  int8_t *zbest;    // [n_total][B]
  int64_t *best;    // [G*B]
  int8_t *zs;       // private scratch, n_max*T per workgroup
  int32_t *nb;
  uint32_t *prio;
  int8_t *fl;
  float *vm;          // momentum, same layout (used when mu != 0)
  int32_t *ls_iters;  // [workgroups]
  int64_t *steps_done;  // [G*B] PGA steps executed, accumulated
  int32_t *err;
};

bool tile_shape_ok(int64_t n_max, int T, int threads, int vec, bool csr_lds, int dreg, int ipt, bool sb);
size_t tile_lds_bytes(int64_t n_max, int T, int64_t nnz_max, bool csr_lds, bool state_lds, bool sb);
hipError_t launch_tile_round(bool maxcut, bool weighted, const TileArgs &a, int threads, hipStream_t s);
// Prop. 4.1 toy: mode 0 = single-coordinate global reset, 1 = full restarts
// (attempts = restarts); n <= 64; x_out [trials][n] or nullptr (mode 0).
void launch_toy(int32_t mode, uint64_t seed, int32_t n, float alpha, float beta, int32_t steps, int32_t attempts,
                int32_t trials, int32_t *first, float *x_out, hipStream_t s);

}  // namespace mqo
