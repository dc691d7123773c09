// libmqo host runtime: argument and graph validation, workspace layout,
// launch plans (persistent tile, batched with hipGraph-captured step
// loops, plain per trajectory), the tile autotuner, and the C-ABI entry
// points declared in include/mqo.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mqo.h"
#include "kernels.h"

using namespace mqo;

namespace {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      return fail(MQO_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                  __LINE__);                                                               \
  } while (0)

#define TRY(expr)               \
  do {                          \
    int _s = (expr);            \
    if (_s != MQO_OK) return _s; \
  } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------------------
// process-wide resources: a private stream (default priority) for blocking
// entry points, pinned readback memory, and plan caches
// ---------------------------------------------------------------------------
// persistent-plan shape: trajectories per workgroup, threads, trajectories
// per lane in the step loop, column indices staged in LDS
struct TileCfg {
  int T, threads, vec, csr, dreg, ipt, sb;  // sb: one iterate buffer (steps gather into registers first)
};

struct Resources {
  std::mutex mu;
  std::mutex host_mu;  // held by the blocking entry points (pinned buffer, internal stream)
  hipStream_t stream = nullptr;
  int32_t *pinned = nullptr;  // 1024 ints
  int64_t *pinned_voff = nullptr;  // staging of vtx_offset for its upload
  size_t pinned_voff_n = 0;
  hipEvent_t input_ready = nullptr;  // caller's stream -> internal stream
  int device = -1;
  int lds_limit = 0;
  std::string gpu;  // architecture and compute-unit count, part of every tuning key
  // autotuner cache: shape key -> chosen launch shape (text), mirrored to the
  // MQO_TUNE_CACHE file when that is set
  std::map<std::string, std::string> tune;
  bool tune_env_loaded = false;
};

Resources &res() {
  static Resources r;
  return r;
}

// hipGetLastError reports the last error any runtime call of this host
// thread returned, including calls the caller made before ours.  Every
// entry point drops such an error before its first launch, so the check
// after its launches sees only its own.
inline void drop_stale_error() { (void)hipGetLastError(); }

int ensure_resources() {
  Resources &r = res();
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (r.device == dev && r.stream) return MQO_OK;
  if (r.stream) {
    (void)hipStreamDestroy(r.stream);
    r.stream = nullptr;
  }
  if (!r.pinned) HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&r.pinned), 1024 * sizeof(int32_t), 0));
  if (!r.input_ready) HIP_TRY(hipEventCreateWithFlags(&r.input_ready, hipEventDisableTiming));
  HIP_TRY(hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking));
  int lds = 0;
  HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  r.lds_limit = lds;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  std::string arch(prop.gcnArchName);
  arch = arch.substr(0, arch.find(':'));
  r.gpu = arch + "x" + std::to_string(prop.multiProcessorCount);
  r.device = dev;
  return MQO_OK;
}

// ---------------------------------------------------------------------------
// autotuner cache.  One entry per line of the text file: key, a tab, value.
// Keys start with the kind of choice (tile, step, plan) and hold the shape
// they were tuned on (graph size range, mean degree, batch, problem, GPU);
// values are the launch shape chosen and the time it measured.
// ---------------------------------------------------------------------------
int parse_tune_file(const char *path, std::map<std::string, std::string> &out) {
  FILE *f = std::fopen(path, "r");
  if (!f) return fail(MQO_ERR_INVALID_ARG, "cannot open tuning cache %s", path);
  char line[1024];
  int lineno = 0, st = MQO_OK;
  std::map<std::string, std::string> got;
  while (std::fgets(line, sizeof(line), f)) {
    ++lineno;
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    if (l.empty() || l[0] == '#') continue;
    const size_t tab = l.find('\t');
    if (tab == std::string::npos || tab == 0 || tab + 1 >= l.size() || l.find('\t', tab + 1) != std::string::npos) {
      st = fail(MQO_ERR_INVALID_ARG, "tuning cache %s line %d: expected key<TAB>value", path, lineno);
      break;
    }
    got[l.substr(0, tab)] = l.substr(tab + 1);
  }
  std::fclose(f);
  if (st == MQO_OK)
    for (auto &kv : got) out[kv.first] = kv.second;
  return st;
}

// with R.mu held: the MQO_TUNE_CACHE file's entries, once per process
void tune_env_load_locked(Resources &R) {
  if (R.tune_env_loaded) return;
  R.tune_env_loaded = true;
  const char *path = std::getenv("MQO_TUNE_CACHE");
  if (path && *path) {
    std::map<std::string, std::string> got;
    FILE *probe = std::fopen(path, "r");
    if (probe) {
      std::fclose(probe);
      if (parse_tune_file(path, got) == MQO_OK) R.tune.insert(got.begin(), got.end());
    }
  }
}

bool tune_get(const std::string &key, std::string *val) {
  Resources &R = res();
  std::lock_guard<std::mutex> lk(R.mu);
  tune_env_load_locked(R);
  auto it = R.tune.find(key);
  if (it == R.tune.end()) return false;
  *val = it->second;
  return true;
}

void tune_put(const std::string &key, const std::string &val) {
  Resources &R = res();
  std::lock_guard<std::mutex> lk(R.mu);
  tune_env_load_locked(R);
  R.tune[key] = val;
  const char *path = std::getenv("MQO_TUNE_CACHE");
  if (path && *path) {
    FILE *f = std::fopen(path, "a");
    if (f) {
      std::fprintf(f, "%s\t%s\n", key.c_str(), val.c_str());
      std::fclose(f);
    }
  }
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
int check_graph_args(const mqo_graph *g, bool need_weight_free) {
  if (!g) return fail(MQO_ERR_INVALID_ARG, "graph is NULL");
  if (g->num_graphs < 1) return fail(MQO_ERR_INVALID_ARG, "num_graphs must be >= 1");
  if (!g->vtx_offset) return fail(MQO_ERR_INVALID_ARG, "vtx_offset is NULL");
  if (g->vtx_offset[0] != 0) return fail(MQO_ERR_INVALID_GRAPH, "vtx_offset[0] must be 0");
  for (int32_t i = 0; i < g->num_graphs; ++i)
    if (g->vtx_offset[i + 1] <= g->vtx_offset[i])
      return fail(MQO_ERR_INVALID_GRAPH, "graph %d has no vertices (vtx_offset must increase)", i);
  if (g->vtx_offset[g->num_graphs] != g->n_total)
    return fail(MQO_ERR_INVALID_GRAPH, "vtx_offset[G] != n_total");
  if (g->n_total < 1 || g->n_total >= (int64_t)1 << 31) return fail(MQO_ERR_INVALID_GRAPH, "n_total out of range");
  if (g->nnz_total < 0 || g->nnz_total >= (int64_t)1 << 31) return fail(MQO_ERR_INVALID_GRAPH, "nnz out of range");
  if (!g->row_ptr) return fail(MQO_ERR_INVALID_ARG, "row_ptr is NULL");
  if (g->nnz_total > 0 && !g->col_idx) return fail(MQO_ERR_INVALID_ARG, "col_idx is NULL");
  if (need_weight_free && g->weight) return fail(MQO_ERR_INVALID_ARG, "the MIS objective takes an unweighted graph");
  if (g->hub_offset) {
    if (g->hub_min_degree < 0) return fail(MQO_ERR_INVALID_ARG, "hub_min_degree must be >= 0");
    if (g->hub_offset[0] != 0) return fail(MQO_ERR_INVALID_GRAPH, "hub_offset[0] must be 0");
    for (int32_t i = 0; i < g->num_graphs; ++i) {
      const int64_t c = g->hub_offset[i + 1] - g->hub_offset[i];
      if (c < 0 || c > g->vtx_offset[i + 1] - g->vtx_offset[i])
        return fail(MQO_ERR_INVALID_GRAPH, "hub_offset of graph %d out of range", i);
    }
    if (g->hub_offset[g->num_graphs] > 0 && !g->hub_rows) return fail(MQO_ERR_INVALID_ARG, "hub_rows is NULL");
  }
  if (g->max_degree < 0) return fail(MQO_ERR_INVALID_ARG, "max_degree must be >= 0 (0 = unknown)");
  return MQO_OK;
}

int check_params(const mqo_params *p, mqo_objective obj) {
  if (!p) return fail(MQO_ERR_INVALID_ARG, "params is NULL");
  if (p->struct_size != sizeof(mqo_params)) return fail(MQO_ERR_INVALID_ARG, "params.struct_size mismatch");
  if (p->batch < 1) return fail(MQO_ERR_INVALID_ARG, "batch must be >= 1");
  if (p->steps_per_round < 0) return fail(MQO_ERR_INVALID_ARG, "steps_per_round must be >= 0");
  if (p->rounds < 1) return fail(MQO_ERR_INVALID_ARG, "rounds must be >= 1");
  if (p->check_every < 0) return fail(MQO_ERR_INVALID_ARG, "check_every must be >= 0");
  if (!(p->alpha > 0.0f) || !std::isfinite(p->alpha)) return fail(MQO_ERR_INVALID_ARG, "alpha must be > 0");
  if (!(p->momentum >= 0.0f && p->momentum < 1.0f)) return fail(MQO_ERR_INVALID_ARG, "momentum must be in [0,1)");
  if (obj == MQO_OBJ_MIS_H && !(p->gamma > 1.0f && std::isfinite(p->gamma)))
    return fail(MQO_ERR_INVALID_ARG, "gamma must be > 1 (Eq. 3)");
  if (obj != MQO_OBJ_MIS_H) {
    // obj: the continuous objective (a solve passes p->maxcut_objective)
    const int f = obj;
    if (f < MQO_OBJ_MAXCUT_FB || f > MQO_OBJ_MAXCUT_FA) return fail(MQO_ERR_INVALID_ARG, "bad maxcut_objective");
    if (f == MQO_OBJ_MAXCUT_FB && !(p->lambda > 0.0f && p->lambda < 2.0f))
      return fail(MQO_ERR_INVALID_ARG, "lambda must be in (0, 2) (Thm. 3.6)");
    if (f == MQO_OBJ_MAXCUT_FP && !(p->lambda > 0.0f && std::isfinite(p->lambda)))
      return fail(MQO_ERR_INVALID_ARG, "lambda must be > 0 for f_P (Eq. 5)");
    if (f != MQO_OBJ_MAXCUT_FB && p->plan == MQO_PLAN_PERSISTENT)
      return fail(MQO_ERR_UNSUPPORTED, "the persistent plan runs h and f_B only");
    if (f != MQO_OBJ_MAXCUT_FB && p->check_every > 0)
      return fail(MQO_ERR_UNSUPPORTED, "check_every is offered for h and f_B only");
  }
  if (!(p->rho >= 0.0 && p->rho < 1.0)) return fail(MQO_ERR_INVALID_ARG, "rho must be in [0, 1)");
  if (!(p->init_sigma >= 0.0f) || !std::isfinite(p->init_sigma))
    return fail(MQO_ERR_INVALID_ARG, "init_sigma must be >= 0");
  if (p->init_mode != MQO_INIT_UNIFORM && p->init_mode != MQO_INIT_DEGREE)
    return fail(MQO_ERR_INVALID_ARG, "bad init_mode");
  if (p->reset_mode != MQO_RESET_ZERO && p->reset_mode != MQO_RESET_FLIP)
    return fail(MQO_ERR_INVALID_ARG, "bad reset_mode");
  if (p->local_search != MQO_LS_NONE && p->local_search != MQO_LS_ONE_FLIP)
    return fail(MQO_ERR_INVALID_ARG, "bad local_search");
  if (p->final_search != MQO_FINAL_NONE && p->final_search != MQO_FINAL_PAIR)
    return fail(MQO_ERR_INVALID_ARG, "bad final_search");
  if (p->restart_every < 0) return fail(MQO_ERR_INVALID_ARG, "restart_every must be >= 0");
  if (p->pool_k < 0 || p->pool_k > 64 || p->pool_k > p->batch)
    return fail(MQO_ERR_INVALID_ARG, "pool_k must be in [0, min(64, batch)]");
  if (p->pool_k > 0 && p->plan == MQO_PLAN_PLAIN)
    return fail(MQO_ERR_UNSUPPORTED, "the pool couples the trajectories of a graph: not on the plain plan");
  if (p->plan < MQO_PLAN_AUTO || p->plan > MQO_PLAN_PERSISTENT) return fail(MQO_ERR_INVALID_ARG, "bad plan");
  if (p->step_vec != 0 && p->step_vec != 1 && p->step_vec != 2 && p->step_vec != 4)
    return fail(MQO_ERR_INVALID_ARG, "step_vec must be 0, 1, 2 or 4");
  if (p->step_lanes < 0 || p->step_lanes > 64 || (p->step_lanes & (p->step_lanes - 1)))
    return fail(MQO_ERR_INVALID_ARG, "step_lanes must be 0 or a power of two <= 64");
  if (p->traj_count < 0 || (p->traj_count > 0 && !p->traj_ids))
    return fail(MQO_ERR_INVALID_ARG, "traj_count must be >= 0, with traj_ids when > 0");
  if (p->traj_count > 0 && p->plan != MQO_PLAN_PLAIN)
    return fail(MQO_ERR_UNSUPPORTED, "a trajectory subset runs on the plain plan only");
  if (p->tile_cols != 0 && (p->tile_cols < 1 || p->tile_cols > 64 || (p->tile_cols & (p->tile_cols - 1))))
    return fail(MQO_ERR_INVALID_ARG, "tile_cols must be 0 or a power of two <= 64");
  if (p->tile_threads != 0 && p->tile_threads != 256 && p->tile_threads != 512 && p->tile_threads != 1024)
    return fail(MQO_ERR_INVALID_ARG, "tile_threads must be 0, 256, 512 or 1024");
  if (p->tile_vec != 0 && p->tile_vec != 1 && p->tile_vec != 2 && p->tile_vec != 4)
    return fail(MQO_ERR_INVALID_ARG, "tile_vec must be 0, 1, 2 or 4");
  if (p->tile_csr < 0 || p->tile_csr > 2) return fail(MQO_ERR_INVALID_ARG, "tile_csr must be 0, 1 or 2");
  if (p->tile_reg < 0 || p->tile_reg > 2) return fail(MQO_ERR_INVALID_ARG, "tile_reg must be 0, 1 or 2");
  if (p->tile_sb < 0 || p->tile_sb > 2) return fail(MQO_ERR_INVALID_ARG, "tile_sb must be 0, 1 or 2");
  if (p->time_budget_s < 0.0) return fail(MQO_ERR_INVALID_ARG, "time_budget_s must be >= 0");
  return MQO_OK;
}

int64_t max_graph_rows(const mqo_graph *g) {
  int64_t m = 0;
  for (int32_t i = 0; i < g->num_graphs; ++i) m = std::max(m, g->vtx_offset[i + 1] - g->vtx_offset[i]);
  return m;
}

// ---------------------------------------------------------------------------
// workspace layout (one layout covers every plan)
// ---------------------------------------------------------------------------
struct Layout {
  size_t X, Xt, V, Z, Zb, NB, PRIO, F, value, best, acc, act, voff, rpat, bestb, dmax, err, reset, tzs, tnb, tprio,
      tfl, tvm, tls, gorder, lsval, pX, pXt, pV, colact, fixedc, steps, pz[2], pv[2], ph[2], chash, ptaken, psrc,
      pbase, solz, solv, choice, total;
};

// K: pool slots per graph (0 = no pool); the pool buffers come last, so the
// other offsets do not depend on K
Layout make_layout(const mqo_graph *g, int32_t B, int32_t K = 0) {
  Layout L{};
  const int64_t n = g->n_total, G = g->num_graphs, nb = n * B;
  const int64_t tiles_elems = G * (int64_t)(B + 63) * max_graph_rows(g);  // tile scratch, any T <= 64
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.X = take(nb * 4);
  L.Xt = take(nb * 4);
  L.V = take(nb * 4);
  L.Z = take(nb);
  L.Zb = take(nb);
  L.NB = take(nb * 4);
  L.PRIO = take(nb * 4);
  L.F = take(nb);
  L.value = take(G * B * 8);
  L.best = take(G * B * 8);
  L.acc = take(3 * (size_t)B * 8);
  L.act = take(64 * 4);
  L.voff = take((G + 1) * 8);
  L.rpat = take((G + 1) * 4);
  L.bestb = take(G * 4);
  L.dmax = take(64);
  L.err = take(64);
  L.reset = take(reset_scratch_bytes(B));
  L.tzs = take(tiles_elems);
  L.tnb = take(tiles_elems * 4);  // also the pair search's tightness bits (8 n_total ceil(B/64) bytes)
  L.tprio = take(tiles_elems * 4);  // also the pair search's SWAP priorities (n_total * B <= tiles_elems)
  L.tfl = take(tiles_elems);
  L.tvm = take(tiles_elems * 4);
  L.tls = take(G * (int64_t)(B + 63) * 4);
  L.gorder = take(G * 4);  // persistent plan: graphs in launch order
  L.lsval = take((size_t)B * 8);  // the searches' discarded values (not the round's)
  L.pX = take(n * 4);  // plain plan: one trajectory as contiguous vectors
  L.pXt = take(n * 4);
  L.pV = take(n * 4);
  L.colact = take(G * B);  // early exit: trajectory still stepping in this round
  L.fixedc = take(B);      // early exit: rounded point fixed (per column of one graph)
  L.steps = take(G * B * 8);  // PGA steps each trajectory executed
  for (int i = 0; i < 2; ++i) {  // pool, double buffered across rounds
    L.pz[i] = take(n * K);
    L.pv[i] = take(G * K * 8);
    L.ph[i] = take(G * K * 8);
  }
  L.chash = take(K ? G * B * 8 : 0);
  L.ptaken = take(K ? G * (K + B) : 0);
  L.psrc = take(G * K * 4);
  L.pbase = take(K ? G * B * 4 : 0);
  L.solz = take(K ? n : 0);  // the pool modes' best set (I_sol / S_sol) and its value
  L.solv = take(K ? G * 8 : 0);
  L.choice = take(K ? G * 4 : 0);
  L.total = o;
  return L;
}

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(reinterpret_cast<char *>(ws) + off);
}

// max_deg: the largest degree if known (a solve measures it), else -1 for
// the caller's hint g->max_degree (0 = unknown)
GraphView view_of(const mqo_graph *g, int32_t i, int32_t max_deg = -1) {
  GraphView v;
  v.row_ptr = g->row_ptr;
  v.col_idx = g->col_idx;
  v.weight = g->weight;
  v.lo = g->vtx_offset[i];
  v.n = g->vtx_offset[i + 1] - g->vtx_offset[i];
  v.hubs = nullptr;
  v.nhub = 0;
  v.hub_deg = 0x7fffffff;
  if (g->hub_offset && g->hub_offset[i + 1] > g->hub_offset[i]) {
    v.hubs = g->hub_rows + g->hub_offset[i];
    v.nhub = (int32_t)(g->hub_offset[i + 1] - g->hub_offset[i]);
    v.hub_deg = g->hub_min_degree;
  }
  // near-regular (mean degree >= 0.9 x max): row pairs of equal degree are
  // the common case
  const int64_t md = max_deg >= 0 ? max_deg : g->max_degree;
  v.pairs = md > 0 && 10 * g->nnz_total >= 9 * g->n_total * md ? 1 : 0;
  v.xcd_local = g->local_rows == 1;
  return v;
}

int read_back_i32(const int32_t *dev, int count, std::vector<int32_t> &out, hipStream_t s) {
  Resources &r = res();
  out.resize(count);
  for (int off = 0; off < count; off += 1024) {
    const int c = std::min(1024, count - off);
    HIP_TRY(hipMemcpyAsync(r.pinned, dev + off, c * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(out.data() + off, r.pinned, c * sizeof(int32_t));
  }
  return MQO_OK;
}

// Several device int32 ranges read back with one synchronisation.
int read_back_many(const std::vector<std::pair<const int32_t *, int>> &parts, std::vector<int32_t> &out,
                   hipStream_t s) {
  Resources &r = res();
  int total = 0;
  for (const auto &pt : parts) total += pt.second;
  if (total > 1024) {  // larger than the pinned buffer: one at a time
    out.clear();
    for (const auto &pt : parts) {
      std::vector<int32_t> o;
      TRY(read_back_i32(pt.first, pt.second, o, s));
      out.insert(out.end(), o.begin(), o.end());
    }
    return MQO_OK;
  }
  int off = 0;
  for (const auto &pt : parts) {
    HIP_TRY(hipMemcpyAsync(r.pinned + off, pt.first, pt.second * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    off += pt.second;
  }
  HIP_TRY(hipStreamSynchronize(s));
  out.assign(r.pinned, r.pinned + total);
  return MQO_OK;
}

// Device-side canonical-form check with one synchronisation: the column
// and hub checks guard their own reads, so they run in the same pass as the
// row_ptr check.  voff_dev must already hold vtx_offset; err_dev has room
// for 4 ints.  When rpat_dev / dmax_dev are given, it also returns the
// row_ptr entries at the graph boundaries (rp, G+1 values) and the largest
// degree (max_deg).
int validate_on_device(const mqo_graph *g, int64_t *voff_dev, int32_t *err_dev, hipStream_t s,
                       int32_t *rpat_dev = nullptr, int32_t *dmax_dev = nullptr, std::vector<int32_t> *rp = nullptr,
                       int32_t *max_deg = nullptr) {
  launch_fill_i32(err_dev, 4, 0, s);
  launch_validate_rows(g->row_ptr, g->n_total, g->nnz_total, err_dev, s);
  if (g->nnz_total > 0)
    launch_validate_cols(g->row_ptr, g->col_idx, g->weight, voff_dev, g->num_graphs, g->n_total, g->nnz_total,
                         err_dev + 1, s);
  const bool hubs = g->hub_offset != nullptr;
  if (hubs) {
    for (int32_t i = 0; i < g->num_graphs; ++i) {
      const int64_t c = g->hub_offset[i + 1] - g->hub_offset[i];
      if (c > 0)
        launch_validate_hubs(g->row_ptr, g->hub_rows + g->hub_offset[i], c, g->vtx_offset[i],
                             g->vtx_offset[i + 1] - g->vtx_offset[i], g->hub_min_degree, err_dev + 2, s);
    }
    launch_count_hubs(g->row_ptr, g->n_total, g->hub_min_degree, err_dev + 3, s);
  }
  std::vector<std::pair<const int32_t *, int>> parts{{err_dev, 4}};
  if (rpat_dev) {
    launch_gather_rowptr(g->row_ptr, voff_dev, g->num_graphs, rpat_dev, s);
    parts.push_back({rpat_dev, g->num_graphs + 1});
  }
  if (dmax_dev) {
    launch_degree_max(g->row_ptr, g->n_total, dmax_dev, s);
    parts.push_back({dmax_dev, 1});
  }
  HIP_TRY(hipGetLastError());
  std::vector<int32_t> e;
  TRY(read_back_many(parts, e, s));
  if (e[0]) return fail(MQO_ERR_INVALID_GRAPH, "row_ptr is not monotone within [0, nnz]");
  if (e[1] & 2) return fail(MQO_ERR_INVALID_GRAPH, "a column index leaves its graph's vertex range");
  if (e[1] & 4) return fail(MQO_ERR_INVALID_GRAPH, "self loop");
  if (e[1] & 8) return fail(MQO_ERR_INVALID_GRAPH, "columns not strictly ascending within a row");
  if (e[1] & 16) return fail(MQO_ERR_INVALID_GRAPH, "adjacency not symmetric");
  if (e[1] & 32) return fail(MQO_ERR_INVALID_GRAPH, "weights not symmetric");
  if (hubs) {
    if (e[2]) return fail(MQO_ERR_INVALID_GRAPH, "a hub_rows entry is out of its graph, not ascending or not a hub");
    if (e[3] != g->hub_offset[g->num_graphs])
      return fail(MQO_ERR_INVALID_GRAPH, "hub_rows lists %lld rows, the graph has %d of degree > %d",
                  (long long)g->hub_offset[g->num_graphs], e[3], g->hub_min_degree);
  }
  if (rp) rp->assign(e.begin() + 4, e.begin() + 5 + g->num_graphs);
  if (max_deg) *max_deg = e.back();
  return MQO_OK;
}

// ---------------------------------------------------------------------------
// the solve
// ---------------------------------------------------------------------------
struct Solve {
  const mqo_graph *g;
  const mqo_params *p;
  mqo_objective obj;
  bool maxcut;  // discrete side (rounding, cut, local search)
  int form;     // continuous objective of the steps (OBJ_* = mqo_objective)
  float param;
  int32_t B, G;
  int64_t n_max;
  std::vector<int64_t> nnz_g;
  int32_t max_deg = 0;  // largest degree of any vertex in the batch
  void *ws;
  Layout L;
  hipStream_t s;
  const float *x0;
  int8_t *Zb = nullptr;    // incumbents [n_total][B]: the caller's traj_best_x when given, else workspace
  int64_t *best = nullptr; // incumbent values [G*B]: the caller's traj_best_value when given, else workspace
  int64_t ls_iters = 0;
  int64_t search_alt = 0;  // pair iterations that applied a move, summed over the pass searches
  StepCfg step_cfg{0, 0};  // streaming plans: the step kernel's launch shape (of the first loop)
  int32_t deferred_tile_wg = 0;  // > 0: the tile counters sit in the pinned buffer after the final sync
  std::vector<int32_t> gorder;   // persistent plan: graphs in launch order (uploaded once, G > 1)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;  // around the step launches
  // MQO_TRACE: HIP events around every phase of the solve, on its stream
  bool tracing = false;
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> phases;

  hipEvent_t phase_begin() {
    hipEvent_t e = nullptr;
    if (tracing && hipEventCreate(&e) == hipSuccess) (void)hipEventRecord(e, s);
    return e;
  }
  void phase_end(int ph, hipEvent_t e0) {
    if (!e0) return;
    hipEvent_t e1 = nullptr;
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return;
    }
    (void)hipEventRecord(e1, s);
    phases.emplace_back(ph, e0, e1);
  }

  int begin_timed(hipEvent_t *e0) {
    HIP_TRY(hipEventCreate(e0));
    HIP_TRY(hipEventRecord(*e0, s));
    return MQO_OK;
  }
  int end_timed(hipEvent_t e0) {
    hipEvent_t e1;
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e1, s));
    timed.push_back({e0, e1});
    return MQO_OK;
  }
  // after the stream is synchronised
  double timed_ms() {
    double total = 0.0;
    for (auto &p : timed) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess) total += ms;
    }
    return total;
  }
  ~Solve() {
    for (auto &p : timed) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    for (auto &p : phases) {
      (void)hipEventDestroy(std::get<1>(p));
      (void)hipEventDestroy(std::get<2>(p));
    }
  }
};

// Phases of a solve reported by MQO_TRACE.
enum Phase { PH_INIT, PH_RESET, PH_STEPS, PH_LOCAL_SEARCH, PH_EVALUATE, PH_POOL, PH_PAIR_SEARCH, PH_TILE, PH_COUNT };
const char *const PHASE_NAMES[PH_COUNT] = {"init",     "reset", "steps",       "local_search",
                                           "evaluate", "pool",  "pair_search", "persistent_rounds"};

// MQO_TRACE unset or "0": off; "1" or "stderr": one JSON line per solve on
// stderr; anything else: a file the line is appended to.
const char *trace_target() {
  const char *t = std::getenv("MQO_TRACE");
  if (!t || !*t || std::strcmp(t, "0") == 0) return nullptr;
  return t;
}

// After the stream is synchronised: per-phase totals of the HIP-event
// times, one JSON line.
void write_trace(Solve &S, int plan, int32_t rounds_done, double wall_ms) {
  const char *target = trace_target();
  if (!target) return;
  double ms[PH_COUNT] = {};
  int64_t cnt[PH_COUNT] = {};
  for (auto &p : S.phases) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, std::get<1>(p), std::get<2>(p)) == hipSuccess) ms[std::get<0>(p)] += t;
    ++cnt[std::get<0>(p)];
  }
  static const char *const plans[] = {"auto", "plain", "batched", "persistent"};
  std::string line = "{\"mqo_trace\": \"solve\", \"problem\": \"";
  line += S.maxcut ? "maxcut" : "mis";
  char buf[512];
  snprintf(buf, sizeof(buf),
           "\", \"plan\": \"%s\", \"graphs\": %d, \"batch\": %d, \"n_total\": %lld, \"nnz_total\": %lld, "
           "\"rounds_executed\": %d, \"wall_ms\": %.4f, \"phases\": {",
           plans[plan], S.G, S.B, (long long)S.g->n_total, (long long)S.g->nnz_total, rounds_done, wall_ms);
  line += buf;
  bool first = true;
  for (int i = 0; i < PH_COUNT; ++i) {
    if (!cnt[i]) continue;
    snprintf(buf, sizeof(buf), "%s\"%s\": {\"ms\": %.4f, \"count\": %lld}", first ? "" : ", ", PHASE_NAMES[i],
             ms[i], (long long)cnt[i]);
    line += buf;
    first = false;
  }
  line += "}}\n";
  const bool to_stderr = std::strcmp(target, "1") == 0 || std::strcmp(target, "stderr") == 0;
  FILE *f = to_stderr ? stderr : std::fopen(target, "a");
  if (!f) return;
  std::fputs(line.c_str(), f);
  if (to_stderr)
    std::fflush(f);
  else
    std::fclose(f);
}

int k_of(const Solve &S, int64_t n) { return (int)std::floor(S.p->rho * (double)n); }

// initial iterate of every graph into X ([n][B]) unless x0 is given
// start: index of the fresh start of the outer loop (0 = the first)
int init_x(Solve &S, float *X, uint64_t start = 0) {
  for (int32_t gi = 0; gi < S.G; ++gi) {
    const GraphView gv = view_of(S.g, gi, S.max_deg);
    if (S.p->init_mode == MQO_INIT_UNIFORM)
      launch_init_uniform(S.maxcut, X, gv.lo, gv.n, S.B, S.B, S.p->seed, (uint64_t)gi * S.B, S.s, start);
    else
      launch_init_degree(S.maxcut, X, S.g->row_ptr, at<int32_t>(S.ws, S.L.dmax), gv.lo, gv.n, S.B, S.B, S.p->seed,
                         (uint64_t)gi * S.B, S.p->init_sigma, S.s, start);
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

// Mean degree of a batch: it only selects kernel shapes (one wavefront per
// row for the searches on dense graphs), never results.
double mean_degree_of(const mqo_graph *g) {
  return (double)g->nnz_total / (double)std::max<int64_t>(1, g->n_total);
}

// 1-flip local search on columns [traj0, traj0+ncols) of one graph (arrays
// at ld).  Iterations are enqueued Q at a time; each one is skipped on the
// device once an earlier one found no positive gain, and the host reads the
// Q flags to decide whether to continue.  Q starts at q_first and doubles
// up to 8: the searches inside the pair searches, which start at or near
// a 1-flip optimum, start at 2 and waste few launches.
int ls_loop(bool maxcut, const GraphView &gv, int64_t nnz_total, double mean_degree, int8_t *Z, int32_t *NB,
            const uint32_t *PRIO, int8_t *F, int32_t *act, int32_t ncols, int32_t ld, hipStream_t s,
            int64_t *iters_out, int q_first = 8);

int ls_core(bool maxcut, const GraphView &gv, int64_t nnz_total, double mean_degree, uint64_t seed, int32_t round,
            int8_t *Z, int32_t *NB, uint32_t *PRIO, int8_t *F, int32_t *act, long long *acc, int64_t *value_scratch,
            int32_t ncols, int32_t ld, uint64_t traj0, hipStream_t s, int64_t *iters_out) {
  // neighbour counts for the current Z (the values computed here are discarded)
  launch_evaluate(maxcut, gv, Z, NB, acc, value_scratch, nullptr, nullptr, ncols, ld, s);
  launch_ls_prio(PRIO, gv.lo, gv.n, ncols, ld, seed, traj0, (uint64_t)round, s);
  return ls_loop(maxcut, gv, nnz_total, mean_degree, Z, NB, PRIO, F, act, ncols, ld, s, iters_out);
}

// The iterations of the 1-flip search on rows gv (NB = A Z and the
// priorities already in place).
int ls_loop(bool maxcut, const GraphView &gv, int64_t nnz_total, double mean_degree, int8_t *Z, int32_t *NB,
            const uint32_t *PRIO, int8_t *F, int32_t *act, int32_t ncols, int32_t ld, hipStream_t s,
            int64_t *iters_out, int q_first) {
  constexpr int QMAX = 8;  // flags in act
  int Q = std::max(1, std::min(q_first, QMAX));
  int64_t iters = 0;
  const int64_t cap = 4 * (gv.n + nnz_total) + 64;  // never reached: every iteration gains
  std::vector<int32_t> flags;
  while (true) {
    launch_fill_i32(act, Q, 0, s);
    for (int q = 0; q < Q; ++q)
      launch_ls_iteration(maxcut, gv, Z, NB, PRIO, F, act + q, q ? act + q - 1 : nullptr, ncols, ld, mean_degree, s);
    HIP_TRY(hipGetLastError());
    TRY(read_back_i32(act, Q, flags, s));
    int done = 0;
    for (int q = 0; q < Q; ++q) {
      if (flags[q])
        ++iters;
      else {
        done = 1;
        break;
      }
    }
    if (done) break;
    if (iters > cap) return fail(MQO_ERR_INTERNAL, "local search did not terminate");
    Q = std::min(2 * Q, QMAX);
  }
  if (iters_out) *iters_out = iters;
  return MQO_OK;
}

// Rows of every graph of a batch as one view (the search kernels only
// follow edges, which stay inside each graph).
GraphView whole_view(const mqo_graph *g) {
  GraphView v{};
  v.row_ptr = g->row_ptr;
  v.col_idx = g->col_idx;
  v.weight = g->weight;
  v.lo = 0;
  v.n = g->n_total;
  v.hubs = nullptr;
  v.nhub = 0;
  v.hub_deg = 0x7fffffff;
  v.pairs = 0;
  v.xcd_local = g->local_rows == 1;
  return v;
}

// Every graph of the batch as one block-diagonal matrix for the sparse
// product: the hub rows of all graphs (each graph's list is ascending and
// the graphs follow each other, so the concatenation is too) and the
// near-regular flag, as view_of gives them per graph.
GraphView batch_view(const mqo_graph *g, int32_t max_deg) {
  GraphView v = whole_view(g);
  if (g->hub_offset && g->hub_offset[g->num_graphs] > 0) {
    v.hubs = g->hub_rows;
    v.nhub = (int32_t)g->hub_offset[g->num_graphs];
    v.hub_deg = g->hub_min_degree;
  }
  v.pairs = view_of(g, 0, max_deg).pairs;
  return v;
}

// OneTwoSwap / OneTwoFlip on all B columns of every graph of g at once: the
// 1-flip search, then pair iterations each followed by the 1-flip search,
// until an iteration applies no move anywhere (columns that are done stay
// unchanged, so each column's result is its own search's).  The priorities
// (purpose LS and SWAP, trajectory g_i * B + c, local vertex index) are
// drawn once.  T0..T2: int32 scratch [n_total][B] each.
// cand_ms (or nullptr): HIP-event time of the candidate launches, summed.
// Which columns a pair search runs on: graphs [g0, g1) (rows `view`, which
// covers exactly those graphs), ncols columns at leading dimension ld, and
// column c of graph gi is trajectory gi * traj_stride + traj_off + c.
struct PairCols {
  GraphView view;
  int32_t g0, g1;
  int64_t traj_stride, traj_off;
  int32_t ncols, ld;
};

PairCols all_cols(const mqo_graph *g, int32_t B) { return PairCols{whole_view(g), 0, g->num_graphs, B, 0, B, B}; }

int pair_core(bool maxcut, const mqo_graph *g, const PairCols &pc, uint64_t seed, int32_t round, int8_t *Z,
              int32_t *NB, uint32_t *PRIO, uint32_t *PRIO_SW, int8_t *F, int32_t *act, long long *acc,
              int64_t *value_scratch, int32_t *T0, int32_t *T1, int32_t *T2, uint32_t *TB, hipStream_t s,
              int64_t *ls_iters, int64_t *alternations, double *cand_ms) {
  const GraphView &all = pc.view;
  const int32_t B = pc.ncols, ld = pc.ld;
  for (int32_t gi = pc.g0; gi < pc.g1; ++gi) {
    const int64_t lo = g->vtx_offset[gi], n = g->vtx_offset[gi + 1] - lo;
    const uint64_t t0 = (uint64_t)(gi * pc.traj_stride + pc.traj_off);
    launch_ls_prio(PRIO, lo, n, B, ld, seed, t0, (uint64_t)round, s);
    launch_swap_prio(PRIO_SW, lo, n, B, ld, seed, t0, (uint64_t)round, s);
  }
  launch_evaluate(maxcut, all, Z, NB, acc, value_scratch, nullptr, nullptr, B, ld, s);  // NB = A Z
  const int64_t cap = 4 * (g->n_total + g->nnz_total) + 64;  // every applied iteration gains
  int64_t alt = 0;
  std::vector<int32_t> flag;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (cand_ms) {
    *cand_ms = 0.0;
    HIP_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
      (void)hipEventDestroy(ev[0]);
      return fail(MQO_ERR_HIP, "hipEventCreate failed");
    }
  }
  int rc = MQO_OK;
  while (rc == MQO_OK) {
    int64_t it = 0;
    rc = ls_loop(maxcut, all, g->nnz_total, mean_degree_of(g), Z, NB, PRIO, F, act, B, ld, s, &it, 2);
    if (rc != MQO_OK) break;
    if (ls_iters) *ls_iters += it;
    launch_fill_i32(act, 1, 0, s);
    if (cand_ms) (void)hipEventRecord(ev[0], s);
    launch_pair_candidates(maxcut, all, Z, NB, PRIO_SW, T0, T1, T2, TB, B, ld, mean_degree_of(g), s);
    if (cand_ms) (void)hipEventRecord(ev[1], s);
    launch_pair_apply(maxcut, all, Z, NB, PRIO_SW, F, T0, T1, T2, act, B, ld, mean_degree_of(g), s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      rc = fail(MQO_ERR_HIP, "pair iteration: %s", hipGetErrorString(e));
      break;
    }
    rc = read_back_i32(act, 1, flag, s);  // synchronises the stream
    if (rc != MQO_OK) break;
    if (cand_ms) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) *cand_ms += ms;
    }
    if (!flag[0]) break;
    if (++alt > cap) rc = fail(MQO_ERR_INTERNAL, "pair search did not terminate");
  }
  if (cand_ms) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
  }
  if (rc == MQO_OK && alternations) *alternations = alt;
  return rc;
}

int run_local_search(Solve &S, const GraphView &gv, int8_t *Z, int32_t *NB, uint32_t *PRIO, int8_t *F, int32_t ncols,
                     int32_t ld, uint64_t traj0, int32_t round, int64_t *iters_out) {
  return ls_core(S.maxcut, gv, S.g->nnz_total, mean_degree_of(S.g), S.p->seed, round, Z, NB, PRIO, F,
                 at<int32_t>(S.ws, S.L.act), at<long long>(S.ws, S.L.acc), at<int64_t>(S.ws, S.L.lsval), ncols, ld,
                 traj0, S.s, iters_out);
}

// steps on one graph, ping-pong X <-> Xt, result back in X
struct StepLoop {
  // captured step chunks: [0] = the chunk between checks (or the whole
  // round), [1] = the shorter last chunk of a round
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  StepCfg cfg{1, 0};  // launch shape of the step kernel (tuned per shape)
  ~StepLoop() {
    for (int i = 0; i < 2; ++i) {
      if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
    }
  }
};

// Launch shapes of the step kernel for ncols columns at leading dimension
// ld: vec columns per lane (dividing ncols and ld), 2^ll lanes per row, up
// to one lane per column group (more columns than lanes x vec take further
// column slices).  Every shape computes the same sums in the same order.
std::vector<StepCfg> step_candidates(int32_t ncols, int32_t ld) {
  std::vector<StepCfg> out;
  for (int vec : {1, 2, 4}) {
    if (vec > 1 && (ncols % vec != 0 || ld % vec != 0 || ncols < 2 * vec)) continue;
    const int32_t groups = (ncols + vec - 1) / vec;
    for (int ll = 0; ll <= 6; ++ll) {
      if (ll > 0 && (1 << (ll - 1)) >= groups) break;
      out.push_back(StepCfg{vec, ll});
    }
  }
  return out;
}

// The step kernel's launch shape for the rows of gv, by timing every
// candidate on X -> Xt (plain steps: the momentum buffer is not touched)
// once per shape key (graph size range, mean degree, columns, objective,
// weights, hubs, GPU); the key's choice is cached.
// step_vec / step_lanes of the parameters (0 = free) narrow the candidates.
int tune_step(Solve &S, const GraphView &gv, int64_t nnz, const float *X, float *Xt, int32_t ncols, int32_t ld,
              StepCfg *out, double *ms_out = nullptr) {
  if (ms_out) *ms_out = -1.0;  // not timed
  std::vector<StepCfg> cands;
  for (const StepCfg &c : step_candidates(ncols, ld))
    if ((!S.p->step_vec || c.vec == S.p->step_vec) && (!S.p->step_lanes || (1 << c.lanes_log2) == S.p->step_lanes))
      cands.push_back(c);
  if (cands.empty())
    return fail(MQO_ERR_INVALID_ARG, "no step shape with %d columns per lane and %d lanes per row for %d columns",
                S.p->step_vec, S.p->step_lanes, ncols);
  const bool fixed = S.p->step_vec || S.p->step_lanes;
  if (cands.size() == 1 || (!fixed && gv.n * (int64_t)ncols < 4096)) {
    *out = fixed ? cands[0] : default_step_cfg(ncols, ld);  // nothing to choose, or too little work to time
    return MQO_OK;
  }
  const double deg = (double)nnz / (double)gv.n;
  char key[256];
  snprintf(key, sizeof(key), "step|%s|%d|%d|%d|%d|%d|%d|%d|%d|%d", res().gpu.c_str(), S.form, gv.weight != nullptr,
           gv.nhub > 0, (int)std::lround(std::log2((double)gv.n) * 2), (int)std::lround(std::log2(deg + 1.0) * 4),
           ncols, ld, S.p->step_vec, S.p->step_lanes);
  std::string cached;
  if (tune_get(key, &cached)) {
    StepCfg c{};
    double ms = 0.0;
    if (std::sscanf(cached.c_str(), "%d %d %lf", &c.vec, &c.lanes_log2, &ms) == 3)
      for (const StepCfg &k : cands)
        if (k.vec == c.vec && k.lanes_log2 == c.lanes_log2) {
          *out = c;
          if (ms_out) *ms_out = ms;
          return MQO_OK;
        }
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MQO_ERR_HIP, "hipEventCreate failed");
  }
  StepCfg best = cands[0];
  double best_t = 1e30;
  int rc = MQO_OK;
  for (const StepCfg &c : cands) {
    launch_pga_step(S.form, gv, X, Xt, nullptr, ncols, ld, c, S.p->alpha, 0.0f, S.param, S.s);  // warm-up
    (void)hipEventRecord(e0, S.s);
    for (int rep = 0; rep < 3; ++rep)
      launch_pga_step(S.form, gv, X, Xt, nullptr, ncols, ld, c, S.p->alpha, 0.0f, S.param, S.s);
    (void)hipEventRecord(e1, S.s);
    const hipError_t e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = fail(MQO_ERR_HIP, "step tuning: %s", hipGetErrorString(hipGetLastError()));
      break;
    }
    if (ms / 3.0 < best_t) {
      best_t = ms / 3.0;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  TRY(rc);
  char val[64];
  snprintf(val, sizeof(val), "%d %d %.6f", best.vec, best.lanes_log2, best_t);
  tune_put(key, val);
  *out = best;
  if (ms_out) *ms_out = best_t;
  return MQO_OK;
}

void enqueue_steps(Solve &S, const GraphView &gv, const StepCfg &cfg, float *X, float *Xt, float *V, int32_t ncols,
                   int32_t ld, int32_t steps, const int8_t *colact) {
  float *a = X, *b = Xt;
  for (int32_t st = 0; st < steps; ++st) {
    launch_pga_step(S.form, gv, a, b, V, ncols, ld, cfg, S.p->alpha, S.p->momentum, S.param, S.s, colact);
    std::swap(a, b);
  }
  if (a != X) launch_copy_f32(a + gv.lo * ld, X + gv.lo * ld, gv.n * ld, S.s);
}

int run_chunk(Solve &S, StepLoop &loop, int slot, bool use_graph, const GraphView &gv, float *X, float *Xt,
              float *V, int32_t ncols, int32_t ld, int32_t steps, const int8_t *colact) {
  if (!use_graph) {
    enqueue_steps(S, gv, loop.cfg, X, Xt, V, ncols, ld, steps, colact);
    HIP_TRY(hipGetLastError());
    return MQO_OK;
  }
  if (!loop.exec[slot]) {
    HIP_TRY(hipStreamBeginCapture(S.s, hipStreamCaptureModeThreadLocal));
    enqueue_steps(S, gv, loop.cfg, X, Xt, V, ncols, ld, steps, colact);
    hipError_t e = hipStreamEndCapture(S.s, &loop.graph[slot]);
    if (e != hipSuccess) return fail(MQO_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    HIP_TRY(hipGraphInstantiate(&loop.exec[slot], loop.graph[slot], nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(loop.exec[slot], S.s));
  return MQO_OK;
}

// The round's PGA steps.  With check_every = c > 0: chunks of c steps, and
// after every chunk but the last the rounded point of every still-active
// trajectory is tested (fixed point of the projected step); fixed ones stop
// stepping for the rest of the round.  colact / steps_ctr: the columns'
// active flags and executed-step counters.
int run_steps(Solve &S, StepLoop &loop, bool use_graph, const GraphView &gv, float *X, float *Xt, float *V,
              int32_t ncols, int32_t ld, int8_t *colact, int64_t *steps_ctr, int8_t *Z, int32_t *NB,
              int64_t *value_scratch) {
  const int32_t steps = S.p->steps_per_round;
  if (steps == 0) return MQO_OK;
  const int32_t c = S.p->check_every;
  if (c <= 0) return run_chunk(S, loop, 0, use_graph, gv, X, Xt, V, ncols, ld, steps, nullptr);
  launch_fill_i8(colact, ncols, 1, S.s);
  for (int32_t done = 0; done < steps;) {
    const int32_t len = std::min(c, steps - done);
    launch_count_steps(colact, steps_ctr, ncols, len, S.s);
    TRY(run_chunk(S, loop, len == c ? 0 : 1, use_graph, gv, X, Xt, V, ncols, ld, len, colact));
    done += len;
    if (done < steps) {
      int8_t *fixed = at<int8_t>(S.ws, S.L.fixedc);
      launch_round(S.maxcut, X, Z, gv.lo, gv.n, ncols, ld, S.s);
      launch_evaluate(S.maxcut, gv, Z, NB, at<long long>(S.ws, S.L.acc), value_scratch, nullptr, fixed, ncols, ld,
                      S.s);
      launch_active_update(colact, fixed, ncols, S.s);
    }
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// one round of one graph on columns [traj0, traj0+ncols); arrays at ld,
// incumbents at Zb (ldb) / best / value (offset to traj0 already)
// colact: the columns' early-exit flags; its address is recorded in the
// captured step loops, so a loop shared by several trajectories (plain
// plan) gets one fixed slot
// Zp / base_slot: the pool this round restarts from (nullptr: incumbents)
// The start of round r of one graph: r = 0 the given start (momentum
// cleared), a fresh start of the outer loop, or the reset of the incumbent
// (or of pool slot base_slot[c] of Zp).
void round_start(Solve &S, const GraphView &gv, int32_t r, float *X, float *V, const int8_t *Zb, int32_t ldb,
                 int32_t ncols, int32_t ld, uint64_t traj0, const int8_t *Zp = nullptr, int32_t ldp = 0,
                 const int32_t *base_slot = nullptr) {
  const bool mom = S.p->momentum != 0.0f;
  const int32_t R = S.p->restart_every;
  hipEvent_t ph = S.phase_begin();
  if (r > 0 && R > 0 && r % R == 0) {
    // a fresh start of the outer loop (Alg. 1-4): the initialisation rule
    // with start index r / R; incumbents (and the pool) carry over
    const uint64_t start = (uint64_t)(r / R);
    if (S.p->init_mode == MQO_INIT_UNIFORM)
      launch_init_uniform(S.maxcut, X, gv.lo, gv.n, ncols, ld, S.p->seed, traj0, S.s, start);
    else
      launch_init_degree(S.maxcut, X, S.g->row_ptr, at<int32_t>(S.ws, S.L.dmax), gv.lo, gv.n, ncols, ld, S.p->seed,
                         traj0, S.p->init_sigma, S.s, start);
    if (mom) launch_fill_f32(V + gv.lo * ld, gv.n * ld, 0.0f, S.s);
  } else if (r > 0) {
    launch_reset(S.maxcut, Zb, ldb, nullptr, X, mom ? V : nullptr, gv.lo, gv.n, ncols, ld, S.p->seed, traj0,
                 (uint64_t)r, k_of(S, gv.n), S.p->reset_mode, at<void>(S.ws, S.L.reset), S.s, Zp, ldp, base_slot);
  } else if (mom) {
    launch_fill_f32(V + gv.lo * ld, gv.n * ld, 0.0f, S.s);
  }
  S.phase_end(r > 0 && !(R > 0 && r % R == 0) ? PH_RESET : PH_INIT, ph);
}

// The round's PGA steps on the rows of gv (one graph, or every graph of the
// batch at once when nothing stops early); steps_ctr: the executed-step
// counters of those ncols_ctr trajectories.
int round_steps(Solve &S, StepLoop &loop, bool use_graph, const GraphView &gv, float *X, float *Xt, float *V,
                int32_t ncols, int32_t ld, int8_t *colact, int64_t *steps_ctr, int64_t ncols_ctr, int8_t *Z,
                int32_t *NB, int64_t *value) {
  if (S.p->steps_per_round <= 0) return MQO_OK;
  const bool mom = S.p->momentum != 0.0f;
  hipEvent_t e0;
  TRY(S.begin_timed(&e0));
  hipEvent_t ph = S.phase_begin();
  TRY(run_steps(S, loop, use_graph, gv, X, Xt, mom ? V : nullptr, ncols, ld, colact, steps_ctr, Z, NB, value));
  if (S.p->check_every <= 0) launch_add_i64(steps_ctr, ncols_ctr, S.p->steps_per_round, S.s);
  S.phase_end(PH_STEPS, ph);
  TRY(S.end_timed(e0));
  return MQO_OK;
}

// The end of round r of one graph: rounding, 1-flip search, exact
// evaluation and acceptance (strict improvement; round 0 initialises).
int round_finish(Solve &S, const GraphView &gv, int32_t r, const float *X, int8_t *Z, int8_t *Zb, int32_t ldb,
                 int32_t *NB, uint32_t *PRIO, int8_t *F, int64_t *value, int64_t *best, int32_t ncols, int32_t ld,
                 uint64_t traj0) {
  hipEvent_t ph = S.phase_begin();
  launch_round(S.maxcut, X, Z, gv.lo, gv.n, ncols, ld, S.s);
  if (S.p->local_search == MQO_LS_ONE_FLIP) {
    int64_t it = 0;
    TRY(run_local_search(S, gv, Z, NB, PRIO, F, ncols, ld, traj0, r, &it));
    S.ls_iters += it;
  }
  S.phase_end(PH_LOCAL_SEARCH, ph);
  ph = S.phase_begin();
  launch_evaluate(S.maxcut, gv, Z, NB, at<long long>(S.ws, S.L.acc), value, nullptr, nullptr, ncols, ld, S.s);
  launch_accept(Z, Zb, value, best, gv.lo, gv.n, ncols, ld, ldb, r == 0, S.s);
  S.phase_end(PH_EVALUATE, ph);
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

// one whole round of one graph (start, steps, end)
int grid_round(Solve &S, StepLoop &loop, bool use_graph, const GraphView &gv, int32_t r, float *X, float *Xt,
               float *V, int8_t *Z, int8_t *Zb, int32_t ldb, int32_t *NB, uint32_t *PRIO, int8_t *F, int64_t *value,
               int64_t *best, int32_t ncols, int32_t ld, uint64_t traj0, int8_t *colact, const int8_t *Zp = nullptr,
               int32_t ldp = 0, const int32_t *base_slot = nullptr) {
  round_start(S, gv, r, X, V, Zb, ldb, ncols, ld, traj0, Zp, ldp, base_slot);
  TRY(round_steps(S, loop, use_graph, gv, X, Xt, V, ncols, ld, colact, at<int64_t>(S.ws, S.L.steps) + traj0, ncols,
                  Z, NB, value));
  return round_finish(S, gv, r, X, Z, Zb, ldb, NB, PRIO, F, value, best, ncols, ld, traj0);
}

int32_t search_round(const Solve &S, int32_t r);
bool pass_ends(const Solve &S, int32_t r);
int search_incumbents(Solve &S, int32_t rnd, int64_t *alternations);
int search_one(Solve &S, const GraphView &gv, int32_t gi, int32_t b, int32_t rnd, int64_t *alternations);
void offer_pool(Solve &S, const int8_t *PZ, const int64_t *PV);
int search_pool_pass(Solve &S, const int8_t *PZ, const int64_t *PV, int32_t rnd, int64_t *alternations);

// Every trajectory runs round 0; with a time budget no later round starts
// after it.  With final_search the pair search closes every pass of the
// outer loop (and a pass the budget cut short).
int solve_batched(Solve &S, int32_t *rounds_done) {
  float *X = at<float>(S.ws, S.L.X), *Xt = at<float>(S.ws, S.L.Xt), *V = at<float>(S.ws, S.L.V);
  int8_t *Z = at<int8_t>(S.ws, S.L.Z), *Zb = S.Zb, *F = at<int8_t>(S.ws, S.L.F);
  int32_t *NB = at<int32_t>(S.ws, S.L.NB);
  uint32_t *PRIO = at<uint32_t>(S.ws, S.L.PRIO);
  int64_t *value = at<int64_t>(S.ws, S.L.value), *best = S.best;
  const int32_t B = S.B;
  if (S.x0)
    HIP_TRY(hipMemcpyAsync(X, S.x0, S.g->n_total * B * sizeof(float), hipMemcpyDeviceToDevice, S.s));
  else
    TRY(init_x(S, X));
  // Without early exit the steps of every graph go in one launch over the
  // block-diagonal batch (each row's sums are those of its own graph), one
  // captured loop per round whatever the number of graphs; with it, each
  // graph steps on its own (its trajectories stop independently).
  const bool whole = S.p->check_every <= 0;
  const bool use_graph = S.p->steps_per_round >= 4 && (whole || S.G <= 16);
  const GraphView bv = batch_view(S.g, S.max_deg);
  StepLoop whole_loop;
  std::vector<StepLoop> loops(whole ? 0 : S.G);
  if (whole)
    TRY(tune_step(S, bv, S.g->nnz_total, X, Xt, B, B, &whole_loop.cfg));
  else
    for (int32_t gi = 0; gi < S.G; ++gi)
      TRY(tune_step(S, view_of(S.g, gi, S.max_deg), S.nnz_g[gi], X, Xt, B, B, &loops[gi].cfg));
  S.step_cfg = whole ? whole_loop.cfg : (S.G ? loops[0].cfg : StepCfg{1, 0});
  const int32_t K = S.p->pool_k;
  const bool search = S.p->final_search == MQO_FINAL_PAIR;
  if (K) {
    launch_fill_i64(at<int64_t>(S.ws, S.L.pv[0]), (int64_t)S.G * K, INT64_MIN, S.s);  // empty pool
    launch_fill_i64(at<int64_t>(S.ws, S.L.solv), S.G, INT64_MIN, S.s);              // no best set yet
    launch_fill_i8(at<int8_t>(S.ws, S.L.solz), S.g->n_total, 0, S.s);
  }
  bool searched = false;  // the last round run closed its pass with the search
  const double t0 = now_s();
  int32_t r = 0;
  int64_t *steps_ctr = at<int64_t>(S.ws, S.L.steps);
  int8_t *colact = at<int8_t>(S.ws, S.L.colact);
  for (r = 0; r < S.p->rounds; ++r) {
    if (r > 0 && S.p->time_budget_s > 0.0) {
      HIP_TRY(hipStreamSynchronize(S.s));
      if (now_s() - t0 >= S.p->time_budget_s) break;
    }
    const int cur = r & 1, nxt = cur ^ 1;
    if (K && r > 0)
      launch_pool_bases(at<int64_t>(S.ws, S.L.pv[cur]), K, S.G, B, S.p->seed, (uint64_t)r,
                        at<int32_t>(S.ws, S.L.pbase), S.s);
    for (int32_t gi = 0; gi < S.G; ++gi) {
      const GraphView gv = view_of(S.g, gi, S.max_deg);
      const int64_t t = (int64_t)gi * B;
      const int8_t *Zp = nullptr;
      int32_t *base = nullptr;
      if (K && r > 0) {
        Zp = at<int8_t>(S.ws, S.L.pz[cur]);
        base = at<int32_t>(S.ws, S.L.pbase) + t;
      }
      round_start(S, gv, r, X, V, Zb, B, B, B, (uint64_t)t, Zp, K, base);
      if (!whole)
        TRY(round_steps(S, loops[gi], use_graph, gv, X, Xt, V, B, B, colact + t, steps_ctr + t, B, Z, NB, value + t));
    }
    if (whole)
      TRY(round_steps(S, whole_loop, use_graph, bv, X, Xt, V, B, B, nullptr, steps_ctr, (int64_t)S.G * B, Z, NB,
                      value));
    for (int32_t gi = 0; gi < S.G; ++gi) {
      const GraphView gv = view_of(S.g, gi, S.max_deg);
      const int64_t t = (int64_t)gi * B;
      TRY(round_finish(S, gv, r, X, Z, Zb, B, NB, PRIO, F, value + t, best + t, B, B, (uint64_t)t));
    }
    if (K) {
      hipEvent_t ph = S.phase_begin();
      launch_pool_update(S.maxcut, Z, B, at<int64_t>(S.ws, S.L.voff), S.G, S.g->n_total, B, K, value,
                         at<unsigned long long>(S.ws, S.L.chash), at<int8_t>(S.ws, S.L.ptaken),
                         at<int8_t>(S.ws, S.L.pz[cur]), at<int64_t>(S.ws, S.L.pv[cur]),
                         at<unsigned long long>(S.ws, S.L.ph[cur]), at<int8_t>(S.ws, S.L.pz[nxt]),
                         at<int64_t>(S.ws, S.L.pv[nxt]), at<unsigned long long>(S.ws, S.L.ph[nxt]),
                         at<int32_t>(S.ws, S.L.psrc), S.s);
      S.phase_end(PH_POOL, ph);
    }
    if (K) offer_pool(S, at<int8_t>(S.ws, S.L.pz[nxt]), at<int64_t>(S.ws, S.L.pv[nxt]));
    searched = false;
    if (search && pass_ends(S, r)) {
      if (K)
        TRY(search_pool_pass(S, at<int8_t>(S.ws, S.L.pz[nxt]), at<int64_t>(S.ws, S.L.pv[nxt]), search_round(S, r),
                             &S.search_alt));
      else
        TRY(search_incumbents(S, search_round(S, r), &S.search_alt));
      searched = true;
    }
  }
  if (search && !searched && r > 0) {  // the time budget cut the last pass short
    const int last = r & 1;            // the pool after round r - 1
    if (K)
      TRY(search_pool_pass(S, at<int8_t>(S.ws, S.L.pz[last]), at<int64_t>(S.ws, S.L.pv[last]),
                           search_round(S, r - 1), &S.search_alt));
    else
      TRY(search_incumbents(S, search_round(S, r - 1), &S.search_alt));
  }
  HIP_TRY(hipGetLastError());
  *rounds_done = r;
  return MQO_OK;
}

int solve_plain(Solve &S, int32_t *rounds_done) {
  // One trajectory at a time on contiguous vectors (ld = 1) with the same
  // kernels; incumbents go straight into column b of Zb ([n][B]).  Every
  // trajectory runs round 0, so every incumbent is written; once the time
  // budget has run out no later round starts.  With final_search the pair
  // search closes every pass of the trajectory's outer loop (and a pass the
  // budget cut short).
  float *X = at<float>(S.ws, S.L.pX), *Xt = at<float>(S.ws, S.L.pXt), *V = at<float>(S.ws, S.L.pV);
  int8_t *Z = at<int8_t>(S.ws, S.L.Z), *Zb = S.Zb, *F = at<int8_t>(S.ws, S.L.F);
  int32_t *NB = at<int32_t>(S.ws, S.L.NB);
  uint32_t *PRIO = at<uint32_t>(S.ws, S.L.PRIO);
  int64_t *value = at<int64_t>(S.ws, S.L.value), *best = S.best;
  const int32_t B = S.B;
  const bool search = S.p->final_search == MQO_FINAL_PAIR;
  const float *start = S.x0;
  if (!start) {
    TRY(init_x(S, at<float>(S.ws, S.L.X)));
    start = at<float>(S.ws, S.L.X);
  }
  const bool use_graph = S.p->steps_per_round >= 4;
  const int64_t *ids = S.p->traj_count > 0 ? S.p->traj_ids : nullptr;
  const int64_t count = ids ? S.p->traj_count : (int64_t)S.G * B;
  if (ids) {  // trajectories that do not run: no incumbent
    launch_fill_i64(best, (int64_t)S.G * B, INT64_MIN, S.s);
    launch_fill_i8(Zb, S.g->n_total * B, 0, S.s);
  }
  const double t0 = now_s();
  int32_t rmax = 0;
  bool out_of_time = false;
  int32_t cur_g = -1;
  GraphView gv{};
  std::unique_ptr<StepLoop> loop;  // the captured step loop serves every trajectory of a graph
  for (int64_t i = 0; i < count; ++i) {
    const int64_t t = ids ? ids[i] : i;
    const int32_t gi = (int32_t)(t / B), b = (int32_t)(t % B);
    if (gi != cur_g) {
      gv = view_of(S.g, gi, S.max_deg);
      loop.reset(new StepLoop);
      loop->cfg = default_step_cfg(1, 1);  // one column: one lane per row
      S.step_cfg = loop->cfg;
      cur_g = gi;
    }
    launch_strided_copy_f32(start, B, b, X, 1, 0, gv.lo, gv.n, S.s);
    int32_t r = 0;
    bool searched = false;
    for (r = 0; r < S.p->rounds; ++r) {
      if (r > 0 && S.p->time_budget_s > 0.0 && !out_of_time) {
        HIP_TRY(hipStreamSynchronize(S.s));
        out_of_time = now_s() - t0 >= S.p->time_budget_s;
      }
      if (r > 0 && out_of_time) break;
      TRY(grid_round(S, *loop, use_graph, gv, r, X, Xt, V, Z, Zb + b, B, NB, PRIO, F, value + t, best + t, 1, 1,
                     (uint64_t)t, at<int8_t>(S.ws, S.L.colact)));
      searched = false;
      if (search && pass_ends(S, r)) {
        TRY(search_one(S, gv, gi, b, search_round(S, r), &S.search_alt));
        searched = true;
      }
    }
    if (search && !searched) TRY(search_one(S, gv, gi, b, search_round(S, r - 1), &S.search_alt));
    rmax = std::max(rmax, r);
  }
  *rounds_done = rmax;
  return MQO_OK;
}

// ---------------------------------------------------------------------------
// persistent tile plan + autotuner
// ---------------------------------------------------------------------------
int tile_lds_budget() {
  const int static_lds = 4 * 64 * 4 + 2 * 64 * 8 + 64 * 4 + 2 * 4 + 256;
  return std::min(res().lds_limit, 160 * 1024) - static_lds;
}

int64_t nnz_max_of(const Solve &S) {
  int64_t m = 0;
  for (int64_t x : S.nnz_g) m = std::max(m, x);
  return m;
}

bool tile_feasible(const Solve &S, const TileCfg &c) {
  return tile_shape_ok(S.n_max, c.T, c.threads, c.vec, c.csr != 0, c.dreg, c.ipt, c.sb != 0) &&
         (int64_t)tile_lds_bytes(S.n_max, c.T, nnz_max_of(S), c.csr != 0, c.dreg > 0, c.sb != 0) <=
             tile_lds_budget();
}

// any shape at all fits (plan selection)
bool tile_possible(const Solve &S) {
  if (S.form != OBJ_H && S.form != OBJ_FB) return false;  // the persistent kernel runs h and f_B
  for (int T = 1; T <= 64; T <<= 1)
    for (int th : {256, 512, 1024})
      for (int sb = 0; sb < 2; ++sb)
        if (tile_feasible(S, TileCfg{T, th, 1, 0, 0, 0, sb})) return true;
  return false;
}

// The persistent plan's launch order of the graphs: largest (stored
// entries) first, so that the last workgroups a CU takes are short ones.
// When the graphs split evenly over the 8 XCDs (an XCD takes a contiguous
// range of graph slots, see the kernel's placement), the sorted graphs are
// dealt to the ranges in snake order, so every XCD gets a like share of the
// work, each range again largest first.  Uploaded once per solve.
int tile_graph_order(Solve &S) {
  if (S.G <= 1 || !S.gorder.empty()) return MQO_OK;
  const int32_t G = S.G;
  std::vector<int32_t> idx(G);
  for (int32_t i = 0; i < G; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return S.nnz_g[x] > S.nnz_g[y]; });
  std::vector<int32_t> o(G);
  if (G % 8 == 0) {
    const int32_t per = G / 8;
    int32_t fill[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t i = 0; i < G; ++i) {
      const int32_t pos = i % 8, bin = ((i / 8) & 1) ? 7 - pos : pos;
      o[bin * per + fill[bin]++] = idx[i];
    }
  } else {
    o = idx;
  }
  HIP_TRY(hipMemcpyAsync(at<int32_t>(S.ws, S.L.gorder), o.data(), (size_t)G * sizeof(int32_t), hipMemcpyHostToDevice,
                         S.s));
  S.gorder = std::move(o);  // kept until the solve ends
  return MQO_OK;
}

TileArgs tile_args(Solve &S, const TileCfg &c, const float *x0) {
  TileArgs a{};
  a.gorder = S.gorder.empty() ? nullptr : at<int32_t>(S.ws, S.L.gorder);
  a.row_ptr = S.g->row_ptr;
  a.col_idx = S.g->col_idx;
  a.weight = S.g->weight;
  a.vtx_off = at<int64_t>(S.ws, S.L.voff);
  a.G = S.G;
  a.B = S.B;
  a.T = c.T;
  a.log2T = 0;
  while ((1 << a.log2T) < c.T) ++a.log2T;
  a.tiles = (S.B + c.T - 1) / c.T;
  a.n_max = (int32_t)S.n_max;
  a.nnz_max = (int32_t)nnz_max_of(S);
  a.vec = c.vec;
  a.csr_lds = c.csr;
  a.dreg = c.dreg;
  a.ipt = c.ipt;
  a.sb = c.sb;
  a.steps = S.p->steps_per_round;
  a.reset_mode = S.p->reset_mode;
  a.ls = S.p->local_search == MQO_LS_ONE_FLIP;
  a.alpha = S.p->alpha;
  a.mu = S.p->momentum;
  a.param = S.param;
  a.rho = S.p->rho;
  a.seed = S.p->seed;
  a.x0 = x0;
  a.zbest = S.Zb;
  a.best = S.best;
  a.zs = at<int8_t>(S.ws, S.L.tzs);
  a.nb = at<int32_t>(S.ws, S.L.tnb);
  a.prio = at<uint32_t>(S.ws, S.L.tprio);
  a.fl = at<int8_t>(S.ws, S.L.tfl);
  a.vm = at<float>(S.ws, S.L.tvm);
  a.ls_iters = at<int32_t>(S.ws, S.L.tls);
  a.err = at<int32_t>(S.ws, S.L.err);
  a.check_every = S.p->check_every;
  a.restart_every = S.p->restart_every;
  a.steps_done = at<int64_t>(S.ws, S.L.steps);
  return a;
}

std::string tile_key(const Solve &S) {
  char buf[256];
  const double deg = (double)S.g->nnz_total / (double)S.g->n_total;
  snprintf(buf, sizeof(buf), "%d|%d|%d|%lld|%d|%d|%d|%d", (int)S.maxcut, S.g->weight != nullptr,
           S.p->momentum != 0.0f, (long long)S.n_max, (int)std::lround(std::log2(deg + 1.0) * 4), S.B, S.G,
           S.p->local_search);
  return buf;
}

// Candidate shapes, honouring tile_cols / tile_threads when the caller fixed them.
std::vector<TileCfg> tile_candidates(const Solve &S) {
  int Tmax = 1;
  while (Tmax < S.B && Tmax < 64) Tmax <<= 1;
  std::vector<TileCfg> out;
  for (int T = 1; T <= Tmax; T <<= 1) {
    if (S.p->tile_cols && T != S.p->tile_cols) continue;
    for (int th : {256, 512, 1024}) {
      if (S.p->tile_threads && th != S.p->tile_threads) continue;
      if (S.p->tile_reg != 1 && S.g->weight == nullptr && S.max_deg <= 16) {
        // register adjacency: degree padded to 3, 4, 8 or 16, 1, 2 or 4 rows per lane
        const int dreg = S.max_deg <= 3 ? 3 : S.max_deg <= 4 ? 4 : S.max_deg <= 8 ? 8 : 16;
        const int64_t need = (S.n_max * T + th - 1) / th;
        const int ipt = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 0;
        const TileCfg c{T, th, 1, 0, dreg, ipt};
        if (ipt && (!S.p->tile_vec || S.p->tile_vec == 1) && S.p->tile_csr != 2 && tile_feasible(S, c))
          out.push_back(c);
      }
      if (S.p->tile_reg == 2) continue;
      for (int vec : {1, 2, 4})
        for (int csr : {1, 0}) {
          if (S.p->tile_vec && vec != S.p->tile_vec) continue;
          if (S.p->tile_csr && csr != S.p->tile_csr - 1) continue;
          for (int sb : {0, 1}) {
            if (S.p->tile_sb && sb != S.p->tile_sb - 1) continue;
            const TileCfg c{T, th, vec, csr, 0, 0, sb};
            if (tile_feasible(S, c)) out.push_back(c);
          }
        }
    }
  }
  return out;
}

// Time one round of up to 32 steps per candidate; keep the fastest.  Every
// candidate computes bit-identical results, so this only affects speed.
// ms_per_step (or nullptr): the chosen shape's time per PGA step.
int tune_tile(Solve &S, const float *x0, TileCfg *out, double *ms_per_step = nullptr) {
  TRY(tile_graph_order(S));
  Resources &R = res();
  char fixed[64];
  snprintf(fixed, sizeof(fixed), "|%d|%d|%d|%d|%d|%d|%d", S.p->tile_cols, S.p->tile_threads, S.p->tile_vec,
           S.p->tile_csr, S.p->tile_reg, S.p->tile_sb, S.max_deg);
  const std::string key = "tile|" + R.gpu + "|" + tile_key(S) + fixed;
  std::string cached;
  if (tune_get(key, &cached)) {
    TileCfg c{};
    double ms = 0.0;
    if (std::sscanf(cached.c_str(), "%d %d %d %d %d %d %d %lf", &c.T, &c.threads, &c.vec, &c.csr, &c.dreg, &c.ipt,
                    &c.sb, &ms) == 8 &&
        tile_feasible(S, c)) {
      *out = c;
      if (ms_per_step) *ms_per_step = ms;
      return MQO_OK;
    }
  }
  const std::vector<TileCfg> cands = tile_candidates(S);
  if (cands.empty()) return fail(MQO_ERR_UNSUPPORTED, "no persistent tile shape fits these graphs");
  TileCfg best_c = cands[0];
  double best_t = 1e30;
  const int tsteps = std::max(1, std::min(S.p->steps_per_round, 64));
  {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const bool mc = S.maxcut, w = S.g->weight != nullptr;
    for (const TileCfg &c : cands) {
      // the shapes differ only in the step loop: time one round of up to 64
      // steps without the local search (which depends on the start point)
      TileArgs a = tile_args(S, c, x0);
      a.r0 = 0;
      a.r1 = 1;
      a.steps = tsteps;
      a.ls = 0;
      float ms = 0.f;
      if (launch_tile_round(mc, w, a, c.threads, S.s) != hipSuccess) continue;  // warm-up
      HIP_TRY(hipEventRecord(e0, S.s));
      for (int rep = 0; rep < 2; ++rep) (void)launch_tile_round(mc, w, a, c.threads, S.s);
      HIP_TRY(hipEventRecord(e1, S.s));
      HIP_TRY(hipEventSynchronize(e1));
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      ms /= 2.0f * (float)tsteps;  // per step
      if (ms < best_t) {
        best_t = ms;
        best_c = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  char val[128];
  snprintf(val, sizeof(val), "%d %d %d %d %d %d %d %.6f", best_c.T, best_c.threads, best_c.vec, best_c.csr,
           best_c.dreg, best_c.ipt, best_c.sb, best_t);
  tune_put(key, val);
  *out = best_c;
  if (ms_per_step) *ms_per_step = best_t;
  return MQO_OK;
}

// the launch covers every round of the solve
bool r0_is_whole(const TileArgs &a, const Solve &S) { return a.r0 == 0 && a.r1 == S.p->rounds; }

int solve_tile(Solve &S, int32_t *rounds_done, TileCfg *used) {
  TRY(tile_graph_order(S));
  const float *x0 = S.x0;
  if (!x0) {
    float *X = at<float>(S.ws, S.L.X);
    TRY(init_x(S, X));
    x0 = X;
  }
  TileCfg cfg{};
  TRY(tune_tile(S, x0, &cfg));
  *used = cfg;
  launch_fill_i64(at<int64_t>(S.ws, S.L.steps), (int64_t)S.G * S.B, 0, S.s);  // the tuner's trials counted too
  launch_fill_i32(at<int32_t>(S.ws, S.L.err), 1, 0, S.s);
  TileArgs a = tile_args(S, cfg, x0);
  const bool mc = S.maxcut, w = S.g->weight != nullptr;
  const int nwg = S.G * a.tiles;
  std::vector<int32_t> lsi;
  int32_t r = 0;
  const bool budget = S.p->time_budget_s > 0.0;
  const int32_t R = S.p->restart_every;
  const int32_t K = S.p->pool_k;
  const int32_t B = S.B;
  const bool search = S.p->final_search == MQO_FINAL_PAIR;
  bool searched = false;  // the last round run closed its pass with the search
  if (K) {
    launch_fill_i64(at<int64_t>(S.ws, S.L.pv[0]), (int64_t)S.G * K, INT64_MIN, S.s);  // empty pool
    launch_fill_i64(at<int64_t>(S.ws, S.L.solv), S.G, INT64_MIN, S.s);              // no best set yet
    launch_fill_i8(at<int8_t>(S.ws, S.L.solz), S.g->n_total, 0, S.s);
    a.zc = at<int8_t>(S.ws, S.L.Z);  // the round's candidates and values, for the pool
    a.vc = at<int64_t>(S.ws, S.L.value);
    a.ldp = K;
  }
  const double t0 = now_s();
  // Without a time budget, fresh starts, searches or the pool the whole
  // solve is one launch.  A budget or the pool (which couples the
  // trajectories of a graph after every round) takes a launch per round;
  // fresh starts (every R rounds) a launch per pass of the outer loop, whose
  // first round starts from the initialisation rule written into x0 just
  // before it; the pair search closing a pass runs between launches.
  for (r = 0; r < S.p->rounds;) {
    if (r > 0 && budget) {
      HIP_TRY(hipStreamSynchronize(S.s));
      if (now_s() - t0 >= S.p->time_budget_s) break;
    }
    int32_t r1 = budget || K ? r + 1 : S.p->rounds;
    if (R > 0) r1 = std::min(r1, (r / R + 1) * R);
    const bool fresh = r > 0 && R > 0 && r % R == 0;
    if (fresh) {
      float *X = at<float>(S.ws, S.L.X);
      TRY(init_x(S, X, (uint64_t)(r / R)));
      a.x0 = X;
    }
    const int cur = r & 1, nxt = cur ^ 1;  // the pool before / after round r
    a.zp = nullptr;
    a.base_slot = nullptr;
    if (K && r > 0 && !fresh) {
      int32_t *base = at<int32_t>(S.ws, S.L.pbase);
      launch_pool_bases(at<int64_t>(S.ws, S.L.pv[cur]), K, S.G, B, S.p->seed, (uint64_t)r, base, S.s);
      a.zp = at<int8_t>(S.ws, S.L.pz[cur]);
      a.base_slot = base;
    }
    a.r0 = r;
    a.r1 = r1;
    hipEvent_t e0;
    TRY(S.begin_timed(&e0));
    hipEvent_t ph = S.phase_begin();
    hipError_t e = launch_tile_round(mc, w, a, cfg.threads, S.s);
    if (e != hipSuccess) return fail(MQO_ERR_HIP, "tile launch: %s", hipGetErrorString(e));
    S.phase_end(PH_TILE, ph);
    TRY(S.end_timed(e0));
    r = a.r1;
    if (r == S.p->rounds && r0_is_whole(a, S) && nwg < 1019) {
      // the whole solve in one launch: read back with the final synchronisation
      Resources &Rs = res();
      HIP_TRY(hipMemcpyAsync(Rs.pinned, a.ls_iters, nwg * sizeof(int32_t), hipMemcpyDeviceToHost, S.s));
      HIP_TRY(hipMemcpyAsync(Rs.pinned + nwg, at<int32_t>(S.ws, S.L.err), sizeof(int32_t), hipMemcpyDeviceToHost,
                             S.s));
      S.deferred_tile_wg = nwg;
    } else {
      TRY(read_back_i32(a.ls_iters, nwg, lsi, S.s));
      int64_t mx = 0;
      for (int32_t x : lsi) mx = std::max<int64_t>(mx, x);
      S.ls_iters += mx;
    }
    if (K) {
      hipEvent_t ph = S.phase_begin();
      launch_pool_update(S.maxcut, at<int8_t>(S.ws, S.L.Z), B, at<int64_t>(S.ws, S.L.voff), S.G, S.g->n_total, B, K,
                         at<int64_t>(S.ws, S.L.value), at<unsigned long long>(S.ws, S.L.chash),
                         at<int8_t>(S.ws, S.L.ptaken), at<int8_t>(S.ws, S.L.pz[cur]), at<int64_t>(S.ws, S.L.pv[cur]),
                         at<unsigned long long>(S.ws, S.L.ph[cur]), at<int8_t>(S.ws, S.L.pz[nxt]),
                         at<int64_t>(S.ws, S.L.pv[nxt]), at<unsigned long long>(S.ws, S.L.ph[nxt]),
                         at<int32_t>(S.ws, S.L.psrc), S.s);
      S.phase_end(PH_POOL, ph);
      offer_pool(S, at<int8_t>(S.ws, S.L.pz[nxt]), at<int64_t>(S.ws, S.L.pv[nxt]));
    }
    searched = false;
    if (search && pass_ends(S, r - 1)) {
      if (K)
        TRY(search_pool_pass(S, at<int8_t>(S.ws, S.L.pz[nxt]), at<int64_t>(S.ws, S.L.pv[nxt]),
                             search_round(S, r - 1), &S.search_alt));
      else
        TRY(search_incumbents(S, search_round(S, r - 1), &S.search_alt));
      searched = true;
    }
  }
  if (search && !searched && r > 0) {  // the time budget cut the last pass short
    const int last = r & 1;            // the pool after round r - 1
    if (K)
      TRY(search_pool_pass(S, at<int8_t>(S.ws, S.L.pz[last]), at<int64_t>(S.ws, S.L.pv[last]),
                           search_round(S, r - 1), &S.search_alt));
    else
      TRY(search_incumbents(S, search_round(S, r - 1), &S.search_alt));
  }
  if (!S.deferred_tile_wg) {
    std::vector<int32_t> err;
    TRY(read_back_i32(at<int32_t>(S.ws, S.L.err), 1, err, S.s));
    if (err[0]) return fail(MQO_ERR_INTERNAL, "local search did not terminate");
  }
  *rounds_done = r;
  return MQO_OK;
}

// Consume the tile counters the persistent plan left in the pinned buffer
// (after a synchronisation), before anything else reads back through it.
int settle_deferred(Solve &S) {
  if (!S.deferred_tile_wg) return MQO_OK;
  HIP_TRY(hipStreamSynchronize(S.s));
  const int32_t *pin = res().pinned;
  int64_t mx = 0;
  for (int32_t i = 0; i < S.deferred_tile_wg; ++i) mx = std::max<int64_t>(mx, pin[i]);
  S.ls_iters += mx;
  const bool bad = pin[S.deferred_tile_wg] != 0;
  S.deferred_tile_wg = 0;
  if (bad) return fail(MQO_ERR_INTERNAL, "local search did not terminate");
  return MQO_OK;
}

// Philox round index of the search closing the pass of the outer loop that
// round r belongs to: rounds + the pass number
int32_t search_round(const Solve &S, int32_t r) {
  const int32_t R = S.p->restart_every;
  return S.p->rounds + (R > 0 ? r / R : 0);
}

// round r is the last of its pass: the R-th of a fresh start, or the last round
bool pass_ends(const Solve &S, int32_t r) {
  const int32_t R = S.p->restart_every;
  return (R > 0 && (r + 1) % R == 0) || r == S.p->rounds - 1;
}

// T: three int32 scratch arrays of [n_total][pc.ld] for the pair
// candidates, whose contents are lost (the streaming plans' iterate buffers:
// the round after a search rewrites them whole, by a reset or a fresh start)
int pair_on(Solve &S, const PairCols &pc, int32_t rnd, int8_t *Z, float *const (&T)[3], int64_t *alternations) {
  int64_t alt = 0;
  hipEvent_t ph = S.phase_begin();
  TRY(pair_core(S.maxcut, S.g, pc, S.p->seed, rnd, Z, at<int32_t>(S.ws, S.L.NB), at<uint32_t>(S.ws, S.L.PRIO),
                at<uint32_t>(S.ws, S.L.tprio), at<int8_t>(S.ws, S.L.F), at<int32_t>(S.ws, S.L.act),
                at<long long>(S.ws, S.L.acc), at<int64_t>(S.ws, S.L.lsval), reinterpret_cast<int32_t *>(T[0]),
                reinterpret_cast<int32_t *>(T[1]), reinterpret_cast<int32_t *>(T[2]), at<uint32_t>(S.ws, S.L.tnb),
                S.s, &S.ls_iters, &alt, nullptr));
  S.phase_end(PH_PAIR_SEARCH, ph);
  *alternations += alt;
  return MQO_OK;
}

// Alg. 1 / Alg. 2, the search closing a pass of the outer loop: the pair
// search on every incumbent (all trajectories of all graphs, round index
// rnd), each replaced when strictly better, so the next pass resets from
// the searched sets.  The iterate buffers and the tile scratch serve as
// scratch.
int search_incumbents(Solve &S, int32_t rnd, int64_t *alternations) {
  TRY(settle_deferred(S));
  int8_t *Z = at<int8_t>(S.ws, S.L.Z), *Zb = S.Zb;
  int64_t *value = at<int64_t>(S.ws, S.L.value), *best = S.best;
  const int32_t B = S.B;
  HIP_TRY(hipMemcpyAsync(Z, Zb, (size_t)S.g->n_total * B, hipMemcpyDeviceToDevice, S.s));
  float *const T[3] = {at<float>(S.ws, S.L.X), at<float>(S.ws, S.L.Xt), at<float>(S.ws, S.L.V)};
  TRY(pair_on(S, all_cols(S.g, B), rnd, Z, T, alternations));
  for (int32_t gi = 0; gi < S.G; ++gi) {
    const GraphView gv = view_of(S.g, gi, S.max_deg);
    const int64_t t = (int64_t)gi * B;
    launch_evaluate(S.maxcut, gv, Z, at<int32_t>(S.ws, S.L.NB), at<long long>(S.ws, S.L.acc), value + t, nullptr,
                    nullptr, B, B, S.s);
    launch_accept(Z, Zb, value + t, best + t, gv.lo, gv.n, B, B, B, false, S.s);
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

// The same for the one trajectory t = gi B + b of the plain plan (its
// incumbent is column b of Zb); column 0 of the Z scratch (ld 1) holds the
// searched copy.  The pair candidates go to the plan's one-trajectory
// vectors: the [n][B] buffer holds every trajectory's start.
int search_one(Solve &S, const GraphView &gv, int32_t gi, int32_t b, int32_t rnd, int64_t *alternations) {
  int8_t *Z = at<int8_t>(S.ws, S.L.Z);
  int64_t *value = at<int64_t>(S.ws, S.L.value);
  const int64_t t = (int64_t)gi * S.B + b;
  launch_strided_copy_i8(S.Zb, S.B, b, Z, 1, 0, gv.lo, gv.n, S.s);
  float *const T[3] = {at<float>(S.ws, S.L.pX), at<float>(S.ws, S.L.pXt), at<float>(S.ws, S.L.pV)};
  TRY(pair_on(S, PairCols{gv, gi, gi + 1, S.B, b, 1, 1}, rnd, Z, T, alternations));
  launch_evaluate(S.maxcut, gv, Z, at<int32_t>(S.ws, S.L.NB), at<long long>(S.ws, S.L.acc), value + t, nullptr,
                  nullptr, 1, 1, S.s);
  launch_accept(Z, S.Zb + b, value + t, S.best + t, gv.lo, gv.n, 1, 1, S.B, false, S.s);
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

// The pool modes' best set I_sol / S_sol takes the pool's best member when
// that is strictly better (after every round; PZ / PV: the pool).
void offer_pool(Solve &S, const int8_t *PZ, const int64_t *PV) {
  const int32_t K = S.p->pool_k;
  launch_offer(PZ, K, PV, PV, K, S.G, false, at<int64_t>(S.ws, S.L.voff), S.g->n_total, at<int64_t>(S.ws, S.L.solv),
               at<int8_t>(S.ws, S.L.solz), at<int32_t>(S.ws, S.L.choice), S.s);
}

// The search closing a pass in the pool modes (round index rnd); the pool
// itself is left as it is.  MIS (Alg. 3): I_sol alone, as trajectory g K,
// replacing it when strictly better.  MaxCut (Alg. 4): every pool member
// (trajectory g K + slot), each offered to S_sol in slot order and taken
// when strictly better.
int search_pool_pass(Solve &S, const int8_t *PZ, const int64_t *PV, int32_t rnd, int64_t *alternations) {
  const int32_t K = S.p->pool_k;
  int8_t *Z = at<int8_t>(S.ws, S.L.Z);
  int64_t *value = at<int64_t>(S.ws, S.L.value);
  int64_t *solv = at<int64_t>(S.ws, S.L.solv);
  const int32_t ncols = S.maxcut ? K : 1;
  if (S.maxcut)
    HIP_TRY(hipMemcpyAsync(Z, PZ, (size_t)S.g->n_total * K, hipMemcpyDeviceToDevice, S.s));
  else
    HIP_TRY(hipMemcpyAsync(Z, at<int8_t>(S.ws, S.L.solz), (size_t)S.g->n_total, hipMemcpyDeviceToDevice, S.s));
  float *const T[3] = {at<float>(S.ws, S.L.X), at<float>(S.ws, S.L.Xt), at<float>(S.ws, S.L.V)};
  TRY(pair_on(S, PairCols{whole_view(S.g), 0, S.G, K, 0, ncols, ncols}, rnd, Z, T, alternations));
  for (int32_t gi = 0; gi < S.G; ++gi) {
    const GraphView gv = view_of(S.g, gi, S.max_deg);
    launch_evaluate(S.maxcut, gv, Z, at<int32_t>(S.ws, S.L.NB), at<long long>(S.ws, S.L.acc),
                    value + (int64_t)gi * ncols, nullptr, nullptr, ncols, ncols, S.s);
  }
  // MIS: a graph with no I_sol yet searched an empty vector, which is not offered
  launch_offer(Z, ncols, value, S.maxcut ? PV : nullptr, ncols, S.G, !S.maxcut, at<int64_t>(S.ws, S.L.voff),
               S.g->n_total, solv, at<int8_t>(S.ws, S.L.solz), at<int32_t>(S.ws, S.L.choice), S.s);
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

// Time a plan on a short copy of the solve: its first min(8, rounds) rounds
// (round 0 from the start point, then rounds from resets, which early exit
// and the search shorten differently on the two plans: the persistent plan's
// workgroups run their rounds independently, the streaming plan's steps wait
// for the slowest trajectory of each round)
// without time budget, pool, fresh starts or final search.  Everything the
// trial writes (incumbents, counters, workspace) the solve writes again; the
// solve's own counters and trace are left as they were.
int trial_plan_ms(Solve &S, int plan, double *ms) {
  mqo_params tp = *S.p;
  tp.rounds = std::min(8, S.p->rounds);
  tp.time_budget_s = 0.0;
  tp.pool_k = 0;
  tp.restart_every = 0;
  tp.final_search = MQO_FINAL_NONE;
  const mqo_params *p0 = S.p;
  const bool tracing0 = S.tracing;
  const int64_t ls0 = S.ls_iters, alt0 = S.search_alt;
  const StepCfg sc0 = S.step_cfg;
  const size_t timed0 = S.timed.size();
  S.p = &tp;
  S.tracing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess ? MQO_OK
                                                                                   : fail(MQO_ERR_HIP, "event create");
  if (st == MQO_OK) {
    (void)hipEventRecord(e0, S.s);
    int32_t rounds_done = 0;
    TileCfg used{};
    st = plan == MQO_PLAN_PERSISTENT ? solve_tile(S, &rounds_done, &used) : solve_batched(S, &rounds_done);
    if (st == MQO_OK) st = settle_deferred(S);
    (void)hipEventRecord(e1, S.s);
    if (st == MQO_OK && hipEventSynchronize(e1) != hipSuccess) st = fail(MQO_ERR_HIP, "trial synchronise");
    float t = 0.0f;
    if (st == MQO_OK) (void)hipEventElapsedTime(&t, e0, e1);
    *ms = t;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (size_t i = timed0; i < S.timed.size(); ++i) {
    (void)hipEventDestroy(S.timed[i].first);
    (void)hipEventDestroy(S.timed[i].second);
  }
  S.timed.resize(timed0);
  S.p = p0;
  S.tracing = tracing0;
  S.ls_iters = ls0;
  S.search_alt = alt0;
  S.step_cfg = sc0;
  return st;
}

// MQO_PLAN_AUTO: the streaming (batched) plan when no persistent tile shape
// fits, else the faster of the two: per PGA step over the whole batch (the
// best persistent tile shape's round of steps against the best streaming
// step launch) when one is more than twice as fast as the other, else per
// solve, both plans timed on up to eight rounds of it (the rounds' other work --
// rounding, search, reset, launches -- then decides).  Timed once per shape
// key and cached.
int choose_plan(Solve &S, int *plan) {
  if (!tile_possible(S)) {
    *plan = MQO_PLAN_BATCHED;
    return MQO_OK;
  }
  const std::string key = "plan|" + res().gpu + "|" + tile_key(S);
  std::string cached;
  if (tune_get(key, &cached)) {
    if (cached.rfind("persistent", 0) == 0) {
      *plan = MQO_PLAN_PERSISTENT;
      return MQO_OK;
    }
    if (cached.rfind("batched", 0) == 0) {
      *plan = MQO_PLAN_BATCHED;
      return MQO_OK;
    }
  }
  float *X = at<float>(S.ws, S.L.X), *Xt = at<float>(S.ws, S.L.Xt);
  if (S.x0)
    HIP_TRY(hipMemcpyAsync(X, S.x0, S.g->n_total * S.B * sizeof(float), hipMemcpyDeviceToDevice, S.s));
  else
    TRY(init_x(S, X));
  TileCfg tc{};
  double tile_ms = -1.0, step_ms = -1.0;
  TRY(tune_tile(S, X, &tc, &tile_ms));
  const GraphView bv = batch_view(S.g, S.max_deg);
  // the streaming step in its default shape first: only when that is within
  // twice the persistent round's time per step are its other shapes timed
  {
    const StepCfg dc = default_step_cfg(S.B, S.B);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    launch_pga_step(S.form, bv, X, Xt, nullptr, S.B, S.B, dc, S.p->alpha, 0.0f, S.param, S.s);
    (void)hipEventRecord(e0, S.s);
    launch_pga_step(S.form, bv, X, Xt, nullptr, S.B, S.B, dc, S.p->alpha, 0.0f, S.param, S.s);
    (void)hipEventRecord(e1, S.s);
    const hipError_t e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(e);
    step_ms = ms;
  }
  if (step_ms < 2.0 * tile_ms) {
    StepCfg sc{};
    double tuned = -1.0;
    TRY(tune_step(S, bv, S.g->nnz_total, X, Xt, S.B, S.B, &sc, &tuned));
    if (tuned >= 0.0) step_ms = std::min(step_ms, tuned);
  }
  *plan = step_ms < tile_ms ? MQO_PLAN_BATCHED : MQO_PLAN_PERSISTENT;
  double trial_p = -1.0, trial_b = -1.0;
  if (step_ms < 2.0 * tile_ms && tile_ms < 2.0 * step_ms) {
    TRY(trial_plan_ms(S, MQO_PLAN_PERSISTENT, &trial_p));
    TRY(trial_plan_ms(S, MQO_PLAN_BATCHED, &trial_b));
    *plan = trial_b < trial_p ? MQO_PLAN_BATCHED : MQO_PLAN_PERSISTENT;
  }
  char val[128];
  snprintf(val, sizeof(val), "%s %.6f %.6f %.3f %.3f", *plan == MQO_PLAN_PERSISTENT ? "persistent" : "batched",
           tile_ms, step_ms, trial_p, trial_b);
  tune_put(key, val);
  return MQO_OK;
}

int solve_common(const mqo_graph *g, const mqo_params *p, const float *x0, mqo_result *r, void *ws, size_t ws_bytes,
                 void *stream, mqo_objective obj) {
  TRY(check_graph_args(g, obj == MQO_OBJ_MIS_H));
  if (!p) return fail(MQO_ERR_INVALID_ARG, "params is NULL");
  TRY(check_params(p, obj == MQO_OBJ_MIS_H ? obj : (mqo_objective)p->maxcut_objective));
  if (!r || !r->best_x || !r->best_value) return fail(MQO_ERR_INVALID_ARG, "result arrays best_x/best_value required");
  for (int32_t i = 0; i < p->traj_count; ++i) {
    const int64_t t = p->traj_ids[i];
    if (t < 0 || t >= (int64_t)g->num_graphs * p->batch || (i > 0 && t <= p->traj_ids[i - 1]))
      return fail(MQO_ERR_INVALID_ARG, "traj_ids must be strictly ascending trajectory ids below G * batch");
  }
  const Layout L = make_layout(g, p->batch, p->pool_k);
  if (!ws || ws_bytes < L.total) return fail(MQO_ERR_WORKSPACE, "workspace needs %zu bytes", L.total);
  TRY(ensure_resources());
  std::lock_guard<std::mutex> host_lock(res().host_mu);
  Resources &R = res();
  hipStream_t s = R.stream;
  drop_stale_error();
  // the internal stream waits for the work the caller has queued on `stream`
  HIP_TRY(hipEventRecord(R.input_ready, reinterpret_cast<hipStream_t>(stream)));
  HIP_TRY(hipStreamWaitEvent(s, R.input_ready, 0));

  const double wall0 = now_s();
  Solve S;
  S.tracing = trace_target() != nullptr;
  S.g = g;
  S.p = p;
  S.obj = obj;
  S.maxcut = obj != MQO_OBJ_MIS_H;
  S.form = S.maxcut ? p->maxcut_objective : (int)MQO_OBJ_MIS_H;
  S.param = S.maxcut ? p->lambda : p->gamma;
  S.B = p->batch;
  S.G = g->num_graphs;
  S.n_max = max_graph_rows(g);
  S.ws = ws;
  S.L = L;
  S.s = s;
  S.x0 = x0;
  S.Zb = r->traj_best_x ? r->traj_best_x : at<int8_t>(ws, L.Zb);
  S.best = r->traj_best_value ? r->traj_best_value : at<int64_t>(ws, L.best);

  int64_t *voff = at<int64_t>(ws, L.voff);
  const size_t nvo = (size_t)g->num_graphs + 1;
  if (R.pinned_voff_n < nvo) {
    if (R.pinned_voff) (void)hipHostFree(R.pinned_voff);
    R.pinned_voff = nullptr;
    R.pinned_voff_n = 0;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&R.pinned_voff), nvo * sizeof(int64_t), 0));
    R.pinned_voff_n = nvo;
  }
  std::memcpy(R.pinned_voff, g->vtx_offset, nvo * sizeof(int64_t));
  HIP_TRY(hipMemcpyAsync(voff, R.pinned_voff, nvo * sizeof(int64_t), hipMemcpyHostToDevice, s));
  std::vector<int32_t> rp;
  TRY(validate_on_device(g, voff, at<int32_t>(ws, L.err), s, at<int32_t>(ws, L.rpat), at<int32_t>(ws, L.dmax), &rp,
                         &S.max_deg));
  S.nnz_g.resize(S.G);
  for (int32_t i = 0; i < S.G; ++i) S.nnz_g[i] = rp[i + 1] - rp[i];

  int plan = p->plan;
  if (plan == MQO_PLAN_AUTO) TRY(choose_plan(S, &plan));
  launch_fill_i64(at<int64_t>(ws, L.steps), (int64_t)S.G * S.B, 0, s);  // after the plan's trial rounds
  int32_t rounds_done = 0;
  TileCfg used{0, 0, 0, 0, 0, 0};
  if (plan == MQO_PLAN_PERSISTENT)
    TRY(solve_tile(S, &rounds_done, &used));
  else if (plan == MQO_PLAN_BATCHED)
    TRY(solve_batched(S, &rounds_done));
  else
    TRY(solve_plain(S, &rounds_done));
  const int32_t K = p->pool_k;
  const int pool_buf = rounds_done & 1;  // the pool after the last round
  int8_t *PZ = K ? at<int8_t>(ws, L.pz[pool_buf]) : nullptr;
  int64_t *PV = K ? at<int64_t>(ws, L.pv[pool_buf]) : nullptr;

  int64_t *best = S.best;
  int32_t *bestb = at<int32_t>(ws, L.bestb);
  if (K) {  // the answer is the best set I_sol / S_sol (-1 and zeros while there is none)
    launch_pick_best(at<int64_t>(ws, L.solv), S.G, 1, r->best_value, bestb, s);
    launch_copy_best_x(at<int8_t>(ws, L.solz), 1, voff, S.G, bestb, r->best_x, g->n_total, s);
    if (r->pool_x) HIP_TRY(hipMemcpyAsync(r->pool_x, PZ, (size_t)g->n_total * K, hipMemcpyDeviceToDevice, s));
    if (r->pool_value)
      HIP_TRY(hipMemcpyAsync(r->pool_value, PV, (size_t)S.G * K * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  } else {
    launch_pick_best(best, S.G, S.B, r->best_value, bestb, s);
    launch_copy_best_x(S.Zb, S.B, voff, S.G, bestb, r->best_x, g->n_total, s);
  }
  // traj_best_value / traj_best_x, when given, held the incumbents all along
  // exact edge updates: sum over trajectories of executed steps x nnz of the graph
  int64_t *eu_dev = at<int64_t>(ws, L.dmax);  // max degree is on the host already
  launch_edge_updates(at<int64_t>(ws, L.steps), at<int32_t>(ws, L.rpat), S.G, S.B, eu_dev, s);
  int64_t *eu_host = reinterpret_cast<int64_t *>(res().pinned + 1020);  // 8-byte aligned, after the tile counters
  HIP_TRY(hipMemcpyAsync(eu_host, eu_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  TRY(settle_deferred(S));
  r->rounds_executed = rounds_done;
  r->steps_executed = (int64_t)rounds_done * p->steps_per_round;
  r->edge_updates = *eu_host;
  r->plan_used = plan;
  r->tile_cols_used = used.T;
  r->tile_threads_used = used.threads;
  r->tile_vec_used = used.vec;
  r->tile_csr_lds_used = used.csr;
  r->tile_reg_degree_used = used.dreg;
  r->tile_single_buffer_used = used.sb;
  r->ls_iterations = S.ls_iters;
  r->step_kernel_ms = S.timed_ms();
  r->step_kernel_launches = (int64_t)S.timed.size();
  r->final_search_alternations = S.search_alt;
  r->step_vec_used = plan == MQO_PLAN_PERSISTENT ? 0 : S.step_cfg.vec;
  r->step_lanes_used = plan == MQO_PLAN_PERSISTENT ? 0 : 1 << S.step_cfg.lanes_log2;
  if (S.tracing) write_trace(S, plan, rounds_done, 1e3 * (now_s() - wall0));
  return MQO_OK;
}

// per-graph helper for the asynchronous entry points
int check_async(const mqo_graph *g, mqo_objective obj, int32_t B) {
  if (obj < MQO_OBJ_MIS_H || obj > MQO_OBJ_MAXCUT_FA) return fail(MQO_ERR_INVALID_ARG, "bad objective");
  TRY(check_graph_args(g, obj == MQO_OBJ_MIS_H));
  if (B < 1) return fail(MQO_ERR_INVALID_ARG, "B must be >= 1");
  return MQO_OK;
}

int check_param(mqo_objective obj, float param) {
  if (obj == MQO_OBJ_MIS_H && !(param > 1.0f && std::isfinite(param)))
    return fail(MQO_ERR_INVALID_ARG, "gamma must be > 1 (Eq. 3)");
  if (obj == MQO_OBJ_MAXCUT_FB && !(param > 0.0f && param < 2.0f))
    return fail(MQO_ERR_INVALID_ARG, "lambda must be in (0, 2) (Thm. 3.6)");
  if (obj == MQO_OBJ_MAXCUT_FP && !(param > 0.0f && std::isfinite(param)))
    return fail(MQO_ERR_INVALID_ARG, "lambda must be > 0 for f_P (Eq. 5)");
  return MQO_OK;
}

int64_t max_graph_hubs(const mqo_graph *g) {
  int64_t m = 0;
  if (g->hub_offset)
    for (int32_t i = 0; i < g->num_graphs; ++i) m = std::max(m, g->hub_offset[i + 1] - g->hub_offset[i]);
  return m;
}

// float64 partial rows of the objective / adjoint kernels of one graph: one
// per row workgroup, one per hub row, then room for the reduction's slices
size_t partial_count(const mqo_graph *g, int32_t B, int32_t copies = 1) {
  const StepCfg cfg = default_step_cfg(B, B);
  const int64_t nblk = (grid_blocks_x(max_graph_rows(g), cfg) + max_graph_hubs(g)) * copies;
  return (size_t)(nblk + reduce_rows(nblk)) * B;
}

// objective and gradient of every graph after validation; part: the float64
// partial rows (partial_count doubles), needed when f_out is requested
int objective_grad_run(const mqo_graph *g, mqo_objective obj, float param, const float *X, int32_t B,
                       const float *scale, double *f_out, float *grad_out, void *part_ws, void *stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  const bool mc = obj != MQO_OBJ_MIS_H;
  const int form = (int)obj;
  const StepCfg cfg = default_step_cfg(B, B);
  for (int32_t gi = 0; gi < g->num_graphs; ++gi) {
    const GraphView gv = view_of(g, gi);
    const float *sc = scale ? scale + (int64_t)gi * B : nullptr;
    double *part = f_out ? reinterpret_cast<double *>(part_ws) : nullptr;
    launch_objective_grad(form, gv, X, sc, grad_out, part, B, B, cfg, param, s);
    if (f_out) launch_reduce_partials(part, spmm_row_blocks(gv, cfg) + gv.nhub, B, f_out + (int64_t)gi * B, false, s);
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

void mqo_params_default(mqo_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(mqo_params);
  p->batch = 1;
  p->steps_per_round = 200;
  p->rounds = 1;
  p->check_every = 0;
  p->alpha = 0.01f;
  p->momentum = 0.0f;
  p->gamma = 2.0f;
  p->lambda = 1e-3f;
  p->rho = 0.05;
  p->init_sigma = 0.0f;
  p->init_mode = MQO_INIT_UNIFORM;
  p->reset_mode = MQO_RESET_ZERO;
  p->local_search = MQO_LS_ONE_FLIP;
  p->plan = MQO_PLAN_AUTO;
  p->seed = 0;
  p->time_budget_s = 0.0;
  p->maxcut_objective = MQO_OBJ_MAXCUT_FB;
  p->final_search = MQO_FINAL_NONE;
  p->pool_k = 0;
  p->restart_every = 0;
}

size_t mqo_workspace_size(const mqo_graph *g, const mqo_params *p, mqo_objective obj) {
  if (check_graph_args(g, obj == MQO_OBJ_MIS_H) != MQO_OK || !p || p->batch < 1) return 0;
  return make_layout(g, p->batch, p->pool_k >= 0 && p->pool_k <= 64 ? p->pool_k : 0).total;
}

int mqo_solve_mis(const mqo_graph *g, const mqo_params *p, const float *x0, mqo_result *r, void *ws,
                  size_t ws_bytes, void *stream) {
  try {
    return solve_common(g, p, x0, r, ws, ws_bytes, stream, MQO_OBJ_MIS_H);
  } catch (...) {
    return fail(MQO_ERR_INTERNAL, "unexpected exception");
  }
}

int mqo_solve_maxcut(const mqo_graph *g, const mqo_params *p, const float *x0, mqo_result *r, void *ws,
                     size_t ws_bytes, void *stream) {
  try {
    return solve_common(g, p, x0, r, ws, ws_bytes, stream, MQO_OBJ_MAXCUT_FB);
  } catch (...) {
    return fail(MQO_ERR_INTERNAL, "unexpected exception");
  }
}

size_t mqo_objective_workspace_size(const mqo_graph *g, int32_t B) {
  if (check_graph_args(g, false) != MQO_OK || B < 1) return 0;
  return align_up(partial_count(g, B) * sizeof(double));
}

int mqo_objective_grad(const mqo_graph *g, mqo_objective obj, float param, const float *X, int32_t B,
                       const float *scale, double *f_out, float *grad_out, void *ws, size_t ws_bytes, void *stream) {
  TRY(check_async(g, obj, B));
  TRY(check_param(obj, param));
  if (!X) return fail(MQO_ERR_INVALID_ARG, "X is NULL");
  if (f_out && (!ws || ws_bytes < mqo_objective_workspace_size(g, B)))
    return fail(MQO_ERR_WORKSPACE, "workspace needs %zu bytes", mqo_objective_workspace_size(g, B));
  return objective_grad_run(g, obj, param, X, B, scale, f_out, grad_out, ws, stream);
}

int mqo_objective_grad_static(const mqo_graph *g, mqo_objective obj, float param, const float *X, int32_t B,
                              const float *scale, double *f_out, float *grad_out, void *stream) {
  TRY(check_async(g, obj, B));
  TRY(check_param(obj, param));
  if (!X) return fail(MQO_ERR_INVALID_ARG, "X is NULL");
  void *ws = nullptr;
  if (f_out) {
    const size_t need = mqo_objective_workspace_size(g, B);
    if (need > MQO_STATIC_SCRATCH_BYTES)
      return fail(MQO_ERR_WORKSPACE, "the partial sums need %zu bytes, above the static scratch of %u bytes", need,
                  (unsigned)MQO_STATIC_SCRATCH_BYTES);
    HIP_TRY(static_scratch_address(&ws));
  }
  return objective_grad_run(g, obj, param, X, B, scale, f_out, grad_out, ws, stream);
}
size_t mqo_unrolled_workspace_size(const mqo_graph *g, int32_t B, int32_t ckpt_every) {
  if (check_graph_args(g, false) != MQO_OK || B < 1 || ckpt_every < 1) return 0;
  const size_t nb = (size_t)g->n_total * B * sizeof(float);
  // the adjoint's float64 partials of one segment's ckpt_every steps, reduced together
  return align_up(nb) * (size_t)(ckpt_every + 3) + align_up(partial_count(g, B, ckpt_every) * sizeof(double));
}

int mqo_pga_unrolled_forward(const mqo_graph *g, mqo_objective obj, float param, float alpha, int32_t K,
                             int32_t ckpt_every, const float *X0, float *ckpt, float *XK, int32_t B, void *ws,
                             size_t ws_bytes, void *stream) {
  TRY(check_async(g, obj, B));
  TRY(check_param(obj, param));
  if (!(alpha > 0.0f) || !std::isfinite(alpha)) return fail(MQO_ERR_INVALID_ARG, "alpha must be > 0");
  if (K < 1 || ckpt_every < 1 || K % ckpt_every)
    return fail(MQO_ERR_INVALID_ARG, "K must be a positive multiple of ckpt_every");
  if (!X0 || !ckpt || !XK) return fail(MQO_ERR_INVALID_ARG, "X0, ckpt and XK are required");
  if (!ws || ws_bytes < mqo_unrolled_workspace_size(g, B, ckpt_every))
    return fail(MQO_ERR_WORKSPACE, "workspace needs %zu bytes", mqo_unrolled_workspace_size(g, B, ckpt_every));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  const bool mc = obj != MQO_OBJ_MIS_H;
  const int form = (int)obj;
  const StepCfg cfg = default_step_cfg(B, B);
  const int64_t nb = g->n_total * B;
  float *W = reinterpret_cast<float *>(ws);
  const int32_t nseg = K / ckpt_every;
  for (int32_t gi = 0; gi < g->num_graphs; ++gi) {
    const GraphView gv = view_of(g, gi);
    launch_copy_f32(X0 + gv.lo * B, ckpt + gv.lo * B, gv.n * B, s);
    for (int32_t j = 0; j < nseg; ++j) {
      // segment j runs x_{jc} -> x_{(j+1)c}; intermediates alternate between
      // the segment's target and W so that the last step lands on the target
      const float *src = ckpt + (int64_t)j * nb;
      float *target = j == nseg - 1 ? XK : ckpt + (int64_t)(j + 1) * nb;
      for (int32_t i = 1; i <= ckpt_every; ++i) {
        float *dst = ((ckpt_every - i) % 2 == 0) ? target : W;
        launch_pga_step(form, gv, src, dst, nullptr, B, B, cfg, alpha, 0.0f, param, s);
        src = dst;
      }
    }
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

int mqo_pga_unrolled_backward(const mqo_graph *g, mqo_objective obj, float param, float alpha, int32_t K,
                              int32_t ckpt_every, const float *ckpt, const float *dL_dXK, float *dL_dX0,
                              double *dL_dalpha, double *dL_dalpha_sum, int32_t B, void *ws, size_t ws_bytes,
                              void *stream) {
  TRY(check_async(g, obj, B));
  TRY(check_param(obj, param));
  if (!(alpha > 0.0f) || !std::isfinite(alpha)) return fail(MQO_ERR_INVALID_ARG, "alpha must be > 0");
  if (K < 1 || ckpt_every < 1 || K % ckpt_every)
    return fail(MQO_ERR_INVALID_ARG, "K must be a positive multiple of ckpt_every");
  if (!ckpt || !dL_dXK || !dL_dX0 || !dL_dalpha) return fail(MQO_ERR_INVALID_ARG, "NULL array argument");
  if (!ws || ws_bytes < mqo_unrolled_workspace_size(g, B, ckpt_every))
    return fail(MQO_ERR_WORKSPACE, "workspace needs %zu bytes", mqo_unrolled_workspace_size(g, B, ckpt_every));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  const bool mc = obj != MQO_OBJ_MIS_H;
  const int form = (int)obj;
  const StepCfg cfg = default_step_cfg(B, B);
  const int64_t nb = g->n_total * B;
  const size_t slot = align_up((size_t)nb * sizeof(float));
  char *base = reinterpret_cast<char *>(ws);
  std::vector<float *> states(ckpt_every);
  for (int32_t i = 1; i < ckpt_every; ++i) states[i] = reinterpret_cast<float *>(base + slot * (i - 1));
  float *lamA = reinterpret_cast<float *>(base + slot * (ckpt_every - 1));
  float *lamB = reinterpret_cast<float *>(base + slot * ckpt_every);
  float *mu = reinterpret_cast<float *>(base + slot * (ckpt_every + 1));
  double *part = reinterpret_cast<double *>(base + slot * (ckpt_every + 2));
  const int32_t nseg = K / ckpt_every;
  for (int32_t gi = 0; gi < g->num_graphs; ++gi) {
    const GraphView gv = view_of(g, gi);
    const int64_t nblk = spmm_row_blocks(gv, cfg) + gv.nhub;
    launch_copy_f32(dL_dXK + gv.lo * B, lamA + gv.lo * B, gv.n * B, s);
    launch_fill_i64(reinterpret_cast<int64_t *>(dL_dalpha + (int64_t)gi * B), B, 0, s);  // +0.0
    float *cur = lamA, *nxt = lamB;
    for (int32_t j = nseg - 1; j >= 0; --j) {
      states[0] = const_cast<float *>(ckpt + (int64_t)j * nb);
      for (int32_t i = 1; i < ckpt_every; ++i)
        launch_pga_step(form, gv, states[i - 1], states[i], nullptr, B, B, cfg, alpha, 0.0f, param, s);
      // the segment's steps write consecutive partial slabs of nblk rows,
      // summed in one fixed-order reduction per segment
      for (int32_t i = ckpt_every - 1; i >= 0; --i) {
        double *slab = part + (int64_t)(ckpt_every - 1 - i) * nblk * B;
        launch_adjoint_step(form, gv, states[i], cur, mu, nxt, slab, B, B, cfg, alpha, param, s);
        std::swap(cur, nxt);
      }
      launch_reduce_partials(part, (int64_t)ckpt_every * nblk, B, dL_dalpha + (int64_t)gi * B, true, s);
    }
    launch_copy_f32(cur + gv.lo * B, dL_dX0 + gv.lo * B, gv.n * B, s);
  }
  if (dL_dalpha_sum) launch_sum_f64(dL_dalpha, (int64_t)g->num_graphs * B, dL_dalpha_sum, s);
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

// ---- building blocks ----

int mqo_init_iterate(const mqo_graph *g, mqo_objective obj, const mqo_params *p, float *X, void *ws, size_t ws_bytes,
                     void *stream) {
  TRY(check_async(g, obj, p ? p->batch : 0));
  TRY(check_params(p, obj));
  if (!X) return fail(MQO_ERR_INVALID_ARG, "X is NULL");
  if (p->init_mode == MQO_INIT_DEGREE && (!ws || ws_bytes < MQO_INIT_WORKSPACE_BYTES))
    return fail(MQO_ERR_WORKSPACE, "the degree initialisation needs %d bytes of workspace", MQO_INIT_WORKSPACE_BYTES);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  const bool mc = obj != MQO_OBJ_MIS_H;
  const int form = (int)obj;
  const int32_t B = p->batch;
  for (int32_t gi = 0; gi < g->num_graphs; ++gi) {
    const GraphView gv = view_of(g, gi);
    if (p->init_mode == MQO_INIT_UNIFORM)
      launch_init_uniform(mc, X, gv.lo, gv.n, B, B, p->seed, (uint64_t)gi * B, s);
    else
      launch_init_degree(mc, X, g->row_ptr, reinterpret_cast<int32_t *>(ws), gv.lo, gv.n, B, B, p->seed,
                         (uint64_t)gi * B, p->init_sigma, s);
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

int mqo_pga_steps(const mqo_graph *g, mqo_objective obj, const mqo_params *p, float *X, float *V, float *tmp,
                  int32_t nsteps, void *stream) {
  TRY(check_async(g, obj, p ? p->batch : 0));
  TRY(check_params(p, obj));
  if (!X || !tmp || nsteps < 0) return fail(MQO_ERR_INVALID_ARG, "X and tmp are required, nsteps >= 0");
  if (p->momentum != 0.0f && !V) return fail(MQO_ERR_INVALID_ARG, "V is required when momentum != 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  const bool mc = obj != MQO_OBJ_MIS_H;
  const int form = (int)obj;
  const int32_t B = p->batch;
  const float param = mc ? p->lambda : p->gamma;
  const StepCfg cfg = default_step_cfg(B, B);
  for (int32_t gi = 0; gi < g->num_graphs; ++gi) {
    const GraphView gv = view_of(g, gi);
    float *a = X, *b = tmp;
    for (int32_t st = 0; st < nsteps; ++st) {
      launch_pga_step(form, gv, a, b, p->momentum != 0.0f ? V : nullptr, B, B, cfg, p->alpha, p->momentum, param, s);
      std::swap(a, b);
    }
    if (a != X) launch_copy_f32(a + gv.lo * B, X + gv.lo * B, gv.n * B, s);
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

int mqo_round_evaluate(const mqo_graph *g, mqo_objective obj, const float *X, int32_t B, int8_t *Z, int64_t *value,
                       int64_t *conflicts, int8_t *fixed, void *ws, size_t ws_bytes, void *stream) {
  TRY(check_async(g, obj, B));
  if (!X || !Z || !value) return fail(MQO_ERR_INVALID_ARG, "X, Z and value are required");
  const Layout L = make_layout(g, B);
  if (!ws || ws_bytes < L.total) return fail(MQO_ERR_WORKSPACE, "workspace needs %zu bytes", L.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  const bool mc = obj != MQO_OBJ_MIS_H;
  const int form = (int)obj;
  for (int32_t gi = 0; gi < g->num_graphs; ++gi) {
    const GraphView gv = view_of(g, gi);
    const int64_t t = (int64_t)gi * B;
    launch_round(mc, X, Z, gv.lo, gv.n, B, B, s);
    launch_evaluate(mc, gv, Z, at<int32_t>(ws, L.NB), at<long long>(ws, L.acc), value + t,
                    conflicts ? conflicts + t : nullptr, fixed ? fixed + t : nullptr, B, B, s);
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

int mqo_local_search(const mqo_graph *g, mqo_objective obj, int32_t B, uint64_t seed, int32_t round, int8_t *Z,
                     int64_t *iterations, void *ws, size_t ws_bytes, void *stream) {
  TRY(check_async(g, obj, B));
  if (!Z) return fail(MQO_ERR_INVALID_ARG, "Z is NULL");
  const Layout L = make_layout(g, B);
  if (!ws || ws_bytes < L.total) return fail(MQO_ERR_WORKSPACE, "workspace needs %zu bytes", L.total);
  TRY(ensure_resources());
  std::lock_guard<std::mutex> host_lock(res().host_mu);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  const bool mc = obj != MQO_OBJ_MIS_H;
  // every graph of the batch at once: the search only follows edges, which
  // stay inside each graph, so a column that is done stays unchanged
  uint32_t *PRIO = at<uint32_t>(ws, L.PRIO);
  for (int32_t gi = 0; gi < g->num_graphs; ++gi) {
    const int64_t lo = g->vtx_offset[gi], n = g->vtx_offset[gi + 1] - lo;
    launch_ls_prio(PRIO, lo, n, B, B, seed, (uint64_t)gi * B, (uint64_t)round, s);
  }
  const GraphView all = whole_view(g);
  int32_t *NB = at<int32_t>(ws, L.NB);
  launch_evaluate(mc, all, Z, NB, at<long long>(ws, L.acc), at<int64_t>(ws, L.value), nullptr, nullptr, B, B, s);
  int64_t it = 0;
  TRY(ls_loop(mc, all, g->nnz_total, mean_degree_of(g), Z, NB, PRIO, at<int8_t>(ws, L.F), at<int32_t>(ws, L.act), B,
              B, s, &it));
  if (iterations) *iterations = it;
  return MQO_OK;
}

int mqo_pair_search(const mqo_graph *g, mqo_objective obj, int32_t B, uint64_t seed, int32_t round, int8_t *Z,
                    int64_t *alternations, double *candidate_kernel_ms, void *ws, size_t ws_bytes, void *stream) {
  TRY(check_async(g, obj, B));
  if (!Z) return fail(MQO_ERR_INVALID_ARG, "Z is NULL");
  const bool mc = obj != MQO_OBJ_MIS_H;
  if (!mc && g->weight) return fail(MQO_ERR_INVALID_ARG, "MIS graphs carry no weights");
  const Layout L = make_layout(g, B);
  if (!ws || ws_bytes < L.total) return fail(MQO_ERR_WORKSPACE, "workspace needs %zu bytes", L.total);
  TRY(ensure_resources());
  std::lock_guard<std::mutex> host_lock(res().host_mu);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  return pair_core(mc, g, all_cols(g, B), seed, round, Z, at<int32_t>(ws, L.NB), at<uint32_t>(ws, L.PRIO),
                   at<uint32_t>(ws, L.tprio), at<int8_t>(ws, L.F), at<int32_t>(ws, L.act), at<long long>(ws, L.acc),
                   at<int64_t>(ws, L.value), at<int32_t>(ws, L.X), at<int32_t>(ws, L.Xt), at<int32_t>(ws, L.V),
                   at<uint32_t>(ws, L.tnb), s, nullptr, alternations, candidate_kernel_ms);
}

int mqo_reset(const mqo_graph *g, mqo_objective obj, int32_t B, uint64_t seed, int32_t round, double rho,
              int32_t mode, const int8_t *Zbest, const uint32_t *keys, float *X, void *ws, size_t ws_bytes,
              void *stream) {
  TRY(check_async(g, obj, B));
  if (!(rho >= 0.0 && rho < 1.0)) return fail(MQO_ERR_INVALID_ARG, "rho must be in [0, 1)");
  if (mode != MQO_RESET_ZERO && mode != MQO_RESET_FLIP) return fail(MQO_ERR_INVALID_ARG, "bad reset mode");
  if (!Zbest || !X) return fail(MQO_ERR_INVALID_ARG, "Zbest and X are required");
  const Layout L = make_layout(g, B);
  if (!ws || ws_bytes < L.total) return fail(MQO_ERR_WORKSPACE, "workspace needs %zu bytes", L.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  drop_stale_error();
  const bool mc = obj != MQO_OBJ_MIS_H;
  const int form = (int)obj;
  for (int32_t gi = 0; gi < g->num_graphs; ++gi) {
    const GraphView gv = view_of(g, gi);
    const int32_t k = (int32_t)std::floor(rho * (double)gv.n);
    launch_reset(mc, Zbest, B, keys, X, nullptr, gv.lo, gv.n, B, B, seed, (uint64_t)gi * B, (uint64_t)round, k, mode,
                 at<void>(ws, L.reset), s);
  }
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

// ---- validation and misc ----

int mqo_toy_reset(uint64_t seed, int32_t n, float alpha, float beta, int32_t steps, int32_t attempts,
                  int32_t trials, int32_t mode, int32_t *first_hit, float *x_out, void *stream) {
  if (n < 1 || n > 64) return fail(MQO_ERR_INVALID_ARG, "n must be in [1, 64]");
  if (!(alpha > 0.0f) || !std::isfinite(alpha)) return fail(MQO_ERR_INVALID_ARG, "alpha must be > 0");
  if (!(beta > 0.0f && beta < 1.0f)) return fail(MQO_ERR_INVALID_ARG, "beta must be in (0, 1)");
  if (steps < 0 || attempts < 0 || trials < 0) return fail(MQO_ERR_INVALID_ARG, "negative count");
  if (mode != MQO_TOY_GLOBAL_RESET && mode != MQO_TOY_FULL_RESTART) return fail(MQO_ERR_INVALID_ARG, "bad mode");
  if (trials == 0) return MQO_OK;
  if (!first_hit) return fail(MQO_ERR_INVALID_ARG, "first_hit is NULL");
  drop_stale_error();
  launch_toy(mode, seed, n, alpha, beta, steps, attempts, trials, first_hit,
             mode == MQO_TOY_GLOBAL_RESET ? x_out : nullptr, reinterpret_cast<hipStream_t>(stream));
  HIP_TRY(hipGetLastError());
  return MQO_OK;
}

int mqo_validate_graph_host(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                            const int32_t *weight) {
  if (n < 1 || n >= (int64_t)1 << 31) return fail(MQO_ERR_INVALID_GRAPH, "n out of range");
  if (nnz < 0 || nnz >= (int64_t)1 << 31) return fail(MQO_ERR_INVALID_GRAPH, "nnz out of range");
  if (!row_ptr || (nnz > 0 && !col_idx)) return fail(MQO_ERR_INVALID_ARG, "NULL array");
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return fail(MQO_ERR_INVALID_GRAPH, "row_ptr must run from 0 to nnz");
  for (int64_t v = 0; v < n; ++v)
    if (row_ptr[v] > row_ptr[v + 1]) return fail(MQO_ERR_INVALID_GRAPH, "row_ptr not monotone at %lld", (long long)v);
  for (int64_t v = 0; v < n; ++v) {
    for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
      const int64_t c = col_idx[j];
      if (c < 0 || c >= n) return fail(MQO_ERR_INVALID_GRAPH, "column out of range in row %lld", (long long)v);
      if (c == v) return fail(MQO_ERR_INVALID_GRAPH, "self loop at %lld", (long long)v);
      if (j > row_ptr[v] && col_idx[j - 1] >= c)
        return fail(MQO_ERR_INVALID_GRAPH, "row %lld not strictly ascending", (long long)v);
    }
  }
  for (int64_t v = 0; v < n; ++v) {
    for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
      const int64_t c = col_idx[j];
      const int32_t *b = col_idx + row_ptr[c], *e = col_idx + row_ptr[c + 1];
      const int32_t *f = std::lower_bound(b, e, (int32_t)v);
      if (f == e || *f != v) return fail(MQO_ERR_INVALID_GRAPH, "edge (%lld,%lld) has no reverse", (long long)v, (long long)c);
      if (weight && weight[f - col_idx] != weight[j])
        return fail(MQO_ERR_INVALID_GRAPH, "weight of (%lld,%lld) not symmetric", (long long)v, (long long)c);
    }
  }
  return MQO_OK;
}

int mqo_validate_graph(const mqo_graph *g, void *stream) {
  TRY(check_graph_args(g, false));
  TRY(ensure_resources());
  std::lock_guard<std::mutex> host_lock(res().host_mu);
  hipStream_t s = res().stream;
  drop_stale_error();
  if (stream) HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  void *buf = nullptr;
  const size_t bytes = align_up((g->num_graphs + 1) * sizeof(int64_t)) + 256;
  HIP_TRY(hipMalloc(&buf, bytes));
  int64_t *voff = reinterpret_cast<int64_t *>(buf);
  int32_t *err = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(buf) + bytes - 256);
  int st = MQO_OK;
  hipError_t e = hipMemcpyAsync(voff, g->vtx_offset, (g->num_graphs + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    st = fail(MQO_ERR_HIP, "hipMemcpyAsync: %s", hipGetErrorString(e));
  else
    st = validate_on_device(g, voff, err, s);
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  return st;
}

const char *mqo_status_string(int status) {
  switch (status) {
    case MQO_OK:
      return "ok";
    case MQO_ERR_INVALID_ARG:
      return "invalid argument";
    case MQO_ERR_INVALID_GRAPH:
      return "invalid graph";
    case MQO_ERR_WORKSPACE:
      return "workspace too small";
    case MQO_ERR_HIP:
      return "HIP runtime error";
    case MQO_ERR_UNSUPPORTED:
      return "unsupported";
    case MQO_ERR_INTERNAL:
      return "internal error";
    default:
      return "unknown status";
  }
}

const char *mqo_last_error(void) { return g_last_error.c_str(); }

int mqo_version(void) { return MQO_VERSION; }

void mqo_clear_caches(void) {
  Resources &r = res();
  std::lock_guard<std::mutex> lk(r.mu);
  r.tune.clear();
}

int mqo_tune_cache_load(const char *path) {
  if (!path) return fail(MQO_ERR_INVALID_ARG, "path is NULL");
  std::map<std::string, std::string> got;
  TRY(parse_tune_file(path, got));
  Resources &r = res();
  std::lock_guard<std::mutex> lk(r.mu);
  for (auto &kv : got) r.tune[kv.first] = kv.second;
  return MQO_OK;
}

int mqo_tune_cache_save(const char *path) {
  if (!path) return fail(MQO_ERR_INVALID_ARG, "path is NULL");
  Resources &r = res();
  std::lock_guard<std::mutex> lk(r.mu);
  FILE *f = std::fopen(path, "w");
  if (!f) return fail(MQO_ERR_INVALID_ARG, "cannot write tuning cache %s", path);
  std::fprintf(f, "# libmqo autotuner cache: key<TAB>value\n");
  for (auto &kv : r.tune) std::fprintf(f, "%s\t%s\n", kv.first.c_str(), kv.second.c_str());
  const bool ok = std::fclose(f) == 0;
  return ok ? MQO_OK : fail(MQO_ERR_INVALID_ARG, "cannot write tuning cache %s", path);
}

int64_t mqo_tune_cache_size(void) {
  Resources &r = res();
  std::lock_guard<std::mutex> lk(r.mu);
  return (int64_t)r.tune.size();
}


}  // extern "C"
