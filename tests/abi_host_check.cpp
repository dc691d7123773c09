// Host-side checks of libmqo's C-ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code: argument and graph
// validation, workspace sizes, parameter defaults and the autotuner cache
// file.  Nothing here reaches a GPU (every call returns before its first
// runtime call).  Exit status 0 when every check holds.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mqo.h"

static int failures = 0;
#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

// canonical CSR of a cycle on n vertices
static void cycle(int n, std::vector<int32_t> &rp, std::vector<int32_t> &ci) {
  rp.assign(n + 1, 0);
  ci.clear();
  for (int v = 0; v < n; ++v) {
    int a = (v + n - 1) % n, b = (v + 1) % n;
    if (a > b) std::swap(a, b);
    ci.push_back(a);
    ci.push_back(b);
    rp[v + 1] = (int32_t)ci.size();
  }
}

int main(int argc, char **argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  std::vector<int32_t> rp, ci;
  cycle(12, rp, ci);
  // host validation: canonical graph accepted, broken ones refused
  CHECK(mqo_validate_graph_host(12, (int64_t)ci.size(), rp.data(), ci.data(), nullptr) == MQO_OK);
  std::vector<int32_t> bad = ci;
  std::swap(bad[0], bad[1]);  // unsorted row
  CHECK(mqo_validate_graph_host(12, (int64_t)bad.size(), rp.data(), bad.data(), nullptr) == MQO_ERR_INVALID_GRAPH);
  bad = ci;
  bad[0] = 0;  // self loop
  CHECK(mqo_validate_graph_host(12, (int64_t)bad.size(), rp.data(), bad.data(), nullptr) == MQO_ERR_INVALID_GRAPH);
  bad = ci;
  bad[3] = 40;  // out of range
  CHECK(mqo_validate_graph_host(12, (int64_t)bad.size(), rp.data(), bad.data(), nullptr) == MQO_ERR_INVALID_GRAPH);
  CHECK(mqo_validate_graph_host(-1, 0, rp.data(), ci.data(), nullptr) != MQO_OK);
  CHECK(std::strlen(mqo_last_error()) > 0);

  // a graph struct with device pointers that are never dereferenced
  int64_t voff[2] = {0, 12};
  mqo_graph g;
  std::memset(&g, 0, sizeof(g));
  g.num_graphs = 1;
  g.vtx_offset = voff;
  g.n_total = 12;
  g.nnz_total = (int64_t)ci.size();
  g.row_ptr = reinterpret_cast<const int32_t *>(0x1000);
  g.col_idx = reinterpret_cast<const int32_t *>(0x1000);
  mqo_params p;
  mqo_params_default(&p);
  CHECK(p.struct_size == sizeof(mqo_params) && p.batch == 1 && p.rounds == 1);
  p.batch = 8;
  CHECK(mqo_workspace_size(&g, &p, MQO_OBJ_MIS_H) > 0);
  CHECK(mqo_objective_workspace_size(&g, 8) > 0);
  CHECK(mqo_unrolled_workspace_size(&g, 8, 5) > 0);
  // parameter errors come back before any GPU call
  mqo_result r;
  std::memset(&r, 0, sizeof(r));
  mqo_params q = p;
  q.gamma = 1.0f;
  CHECK(mqo_solve_mis(&g, &q, nullptr, &r, nullptr, 0, nullptr) == MQO_ERR_INVALID_ARG);
  q = p;
  q.lambda = 2.5f;
  CHECK(mqo_solve_maxcut(&g, &q, nullptr, &r, nullptr, 0, nullptr) == MQO_ERR_INVALID_ARG);
  q = p;
  q.struct_size = 3;
  CHECK(mqo_solve_mis(&g, &q, nullptr, &r, nullptr, 0, nullptr) == MQO_ERR_INVALID_ARG);
  int64_t ids[2] = {3, 1};
  q = p;
  q.plan = MQO_PLAN_PLAIN;
  q.traj_count = 2;
  q.traj_ids = ids;
  r.best_x = reinterpret_cast<int8_t *>(0x1000);
  r.best_value = reinterpret_cast<int64_t *>(0x1000);
  CHECK(mqo_solve_mis(&g, &q, nullptr, &r, nullptr, 0, nullptr) == MQO_ERR_INVALID_ARG);
  ids[0] = 1;
  ids[1] = 3;
  CHECK(mqo_solve_mis(&g, &q, nullptr, &r, nullptr, 0, nullptr) == MQO_ERR_WORKSPACE);
  // the entry points without a workspace check their own limits on the host
  q = p;
  q.init_mode = MQO_INIT_DEGREE;
  CHECK(mqo_init_iterate(&g, MQO_OBJ_MIS_H, &q, reinterpret_cast<float *>(0x1000), nullptr, 0, nullptr) ==
        MQO_ERR_WORKSPACE);
  std::vector<int64_t> big_off = {0, 400000};
  mqo_graph gb = g;
  gb.vtx_offset = big_off.data();
  gb.n_total = 400000;
  gb.nnz_total = 800000;
  CHECK(mqo_objective_grad_static(&gb, MQO_OBJ_MAXCUT_FB, 1e-3f, reinterpret_cast<const float *>(0x1000), 256,
                                  nullptr, reinterpret_cast<double *>(0x1000), nullptr, nullptr) == MQO_ERR_WORKSPACE);
  for (int st = -6; st <= 0; ++st) CHECK(mqo_status_string(st) != nullptr);

  // autotuner cache: load, save, reload, refuse a malformed file
  mqo_clear_caches();
  const std::string in = dir + "/tune_in.txt", out = dir + "/tune_out.txt", badf = dir + "/tune_bad.txt";
  FILE *f = std::fopen(in.c_str(), "w");
  CHECK(f != nullptr);
  if (f) {
    std::fprintf(f, "# comment\nstep|gfx950x256|0|0|0|14|13|32|32|0|0\t4 3 0.0512\n\nplan|k\tpersistent 1 2\n");
    std::fclose(f);
  }
  CHECK(mqo_tune_cache_load(in.c_str()) == MQO_OK);
  CHECK(mqo_tune_cache_size() == 2);
  CHECK(mqo_tune_cache_save(out.c_str()) == MQO_OK);
  mqo_clear_caches();
  CHECK(mqo_tune_cache_size() == 0);
  CHECK(mqo_tune_cache_load(out.c_str()) == MQO_OK);
  CHECK(mqo_tune_cache_size() == 2);
  f = std::fopen(badf.c_str(), "w");
  if (f) {
    std::fprintf(f, "a\tb\n");
    for (int i = 0; i < 2000; ++i) std::fputc('x', f);  // a line longer than the reader's buffer
    std::fprintf(f, "\nno tab\n");
    std::fclose(f);
  }
  CHECK(mqo_tune_cache_load(badf.c_str()) == MQO_ERR_INVALID_ARG);
  CHECK(mqo_tune_cache_size() == 2);
  CHECK(mqo_tune_cache_load((dir + "/missing.txt").c_str()) == MQO_ERR_INVALID_ARG);
  mqo_clear_caches();
  std::printf("abi host checks: %d failure(s)\n", failures);
  return failures ? 1 : 0;
}
