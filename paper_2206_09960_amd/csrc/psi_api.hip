// extern "C" entry points of the Power-ψ library (declared in include/psi.h).
#include <cstring>
#include <exception>
#include <memory>
#include <new>

#include "psi_internal.h"
#include "psi_tools.h"

namespace psi {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

psi_status step(psi_operator* op, int precision, const double* s_in, double* s_out,
                double* gap_out, int tile_items, int col_segments, int seg_form,
                hipStream_t st);
psi_status final_psi(psi_operator* op, const double* s_vec, double* psi_out, hipStream_t st);
psi_status pass_time(psi_operator* op, int kind, int reps, int tile_items, int col_segments,
                     int seg_form, double* mean_ms, hipStream_t st);

static psi_status check_device(const psi_operator* op) {
  int dev = -1;
  PSI_HIP_CHECK(hipGetDevice(&dev));
  if (dev != op->device) {
    set_error("the current device is not the one the operator was built on");
    return PSI_EINVAL;
  }
  return PSI_OK;
}

}  // namespace psi

using psi::set_error;

#define PSI_GUARD_BEGIN \
  psi::clear_error();   \
  try {
#define PSI_GUARD_END                          \
  }                                            \
  catch (const std::bad_alloc&) {              \
    set_error("host allocation failed");       \
    return PSI_EDEVICE;                        \
  }                                            \
  catch (const std::exception& e) {            \
    set_error(e.what());                       \
    return PSI_EDEVICE;                        \
  }                                            \
  catch (...) {                                \
    set_error("unknown C++ exception");        \
    return PSI_EDEVICE;                        \
  }

extern "C" {

const char* psi_version(void) { return "psi-mi355x 0.1 (gfx950)"; }

const char* psi_last_error(void) { return psi::g_last_error.c_str(); }

psi_status psi_operator_workspace_size(int64_t n_users, int64_t n_edges, int32_t n_graphs,
                                       uint32_t flags, size_t* persistent_bytes,
                                       size_t* scratch_bytes) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(n_users >= 1 && n_users < (int64_t(1) << 30), "n_users must be in [1, 2^30)");
  PSI_REQUIRE(n_edges >= 0, "n_edges must be >= 0");
  PSI_REQUIRE(n_users + n_edges < (int64_t(1) << 31) - 4096, "n_users + n_edges too large");
  PSI_REQUIRE(n_graphs >= 1, "n_graphs must be >= 1");
  PSI_REQUIRE(persistent_bytes && scratch_bytes, "output pointers must not be NULL");
  psi::Layout L = psi::compute_layout(n_users, n_edges, n_graphs, flags);
  *persistent_bytes = L.persistent;
  *scratch_bytes = L.scratch;
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_build_operator(int64_t n_users, int64_t n_edges, const int32_t* follower,
                              const int32_t* leader, const double* lambda, const double* mu,
                              int32_t n_graphs, const int64_t* node_offsets, uint32_t flags,
                              void* persistent, size_t persistent_bytes, void* scratch,
                              size_t scratch_bytes, void* stream, psi_operator** op) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  *op = nullptr;
  PSI_REQUIRE(n_users >= 1 && n_users < (int64_t(1) << 30), "n_users must be in [1, 2^30)");
  PSI_REQUIRE(n_edges >= 0, "n_edges must be >= 0");
  PSI_REQUIRE(n_users + n_edges < (int64_t(1) << 31) - 4096, "n_users + n_edges too large");
  PSI_REQUIRE(n_edges == 0 || (follower && leader), "edge arrays must not be NULL");
  PSI_REQUIRE(lambda && mu, "lambda and mu must not be NULL");
  PSI_REQUIRE(n_graphs >= 1, "n_graphs must be >= 1");
  PSI_REQUIRE(persistent && scratch, "workspaces must not be NULL");
  if (n_graphs > 1) {
    PSI_REQUIRE(n_graphs < 65536, "at most 65535 graphs");
    PSI_REQUIRE(node_offsets, "node_offsets needed when n_graphs > 1");
    PSI_REQUIRE(node_offsets[0] == 0 && node_offsets[n_graphs] == n_users,
                "node_offsets must run from 0 to n_users");
    for (int g = 0; g < n_graphs; ++g)
      PSI_REQUIRE(node_offsets[g + 1] > node_offsets[g], "every graph needs at least one user");
  }
  psi::Layout L = psi::compute_layout(n_users, n_edges, n_graphs, flags);
  if (persistent_bytes < L.persistent || scratch_bytes < L.scratch) {
    set_error("workspace smaller than psi_operator_workspace_size reported");
    return PSI_ENOSPACE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  // owned here until the build succeeds, so early returns and exceptions free it
  std::unique_ptr<psi_operator> o(new psi_operator());
  PSI_HIP_CHECK(hipGetDevice(&o->device));
  o->n = n_users;
  o->m_in = n_edges;
  o->n_graphs = n_graphs;
  o->flags = flags;
  if (n_graphs > 1) o->node_offsets.assign(node_offsets, node_offsets + n_graphs + 1);
  else o->node_offsets = {0, n_users};
  psi::carve_persistent(o.get(), static_cast<char*>(persistent), n_edges, n_graphs);
  psi_status s = psi::build_operator(o.get(), follower, leader, lambda, mu, node_offsets,
                                     static_cast<char*>(scratch), scratch_bytes, st);
  if (s == PSI_OK) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&o->host_ctrl), 2 * sizeof(psi::Ctrl),
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
      set_error(std::string("hipHostMalloc: ") + hipGetErrorString(e));
      s = PSI_EDEVICE;
    }
  }
  if (s != PSI_OK) {
    if (o->host_ctrl) (void)hipHostFree(o->host_ctrl);
    return s;
  }
  *op = o.release();
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_operator_destroy(psi_operator* op) {
  PSI_GUARD_BEGIN
  if (!op) return PSI_OK;
  if (op->host_ctrl) (void)hipHostFree(op->host_ctrl);
  delete op;
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_operator_get_stats(const psi_operator* op, psi_operator_stats* out) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op && out, "arguments must not be NULL");
  *out = op->stats;
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_operator_views(const psi_operator* op, const int32_t** row_ptr,
                              const int32_t** col, const double** c, const double** d,
                              const double** inv_den) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  if (row_ptr) *row_ptr = op->row_ptr;
  if (col) *col = op->col;
  if (c) *c = op->c;
  if (d) *d = op->d;
  if (inv_den) *inv_den = op->invden;
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_params_default(psi_params* p) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(p, "p must not be NULL");
  std::memset(p, 0, sizeof(*p));
  p->tol = 1e-8;
  p->tol_mode = PSI_TOL_ABS_L1;
  p->max_iter = 10000;
  p->precision = PSI_PREC_FP64;
  p->check_every = 0;
  p->flags = 0;
  p->tile_items = 0;
  p->col_segments = 0;
  p->seg_form = 0;
  p->inner_tol = 0.0;
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_solve(psi_operator* op, const psi_params* prm, const double* s0,
                     double* psi_out, double* s_out, psi_info* info, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status s = psi::check_device(op);
  if (s != PSI_OK) return s;
  return psi::solve(op, prm, s0, psi_out, s_out, info, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_solve_async(psi_operator* op, const psi_params* prm, const double* s0,
                           double* psi_out, double* s_out, psi_info* info, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status s = psi::check_device(op);
  if (s != PSI_OK) return s;
  return psi::solve_async(op, prm, s0, psi_out, s_out, info, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_pagerank(psi_operator* op, double alpha, const psi_params* prm,
                        int32_t power_method, double* start, double* pi_out, psi_info* info,
                        void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status s = psi::check_device(op);
  if (s != PSI_OK) return s;
  return psi::pagerank(op, alpha, prm, power_method, start, pi_out, info,
                       static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_step(psi_operator* op, int32_t precision, const double* s_in, double* s_out,
                    double* gap_out, int32_t tile_items, int32_t col_segments,
                    int32_t seg_form, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status s = psi::check_device(op);
  if (s != PSI_OK) return s;
  return psi::step(op, precision, s_in, s_out, gap_out, tile_items, col_segments, seg_form,
                   static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_final(psi_operator* op, const double* s, double* psi_out, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  PSI_REQUIRE(op->n_graphs == 1, "psi_final: multi-graph operators are finished by psi_solve_batched");
  psi_status st = psi::check_device(op);
  if (st != PSI_OK) return st;
  return psi::final_psi(op, s, psi_out, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_operator_band_info(const psi_operator* op, int32_t* col_log, int32_t* rows,
                                  int32_t* col_blocks, int32_t* row_blocks, int32_t* bands,
                                  int32_t* split_rows) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "operator must not be NULL");
  const bool b = op->band_built;
  if (col_log) *col_log = b ? op->band_wlog : 0;
  if (rows) *rows = b ? op->band_rows : 0;
  if (col_blocks) *col_blocks = b ? op->band_B : 0;
  if (row_blocks) *row_blocks = b ? op->band_nb : 0;
  if (bands) *bands = b ? op->band_count : 0;
  if (split_rows) *split_rows = b ? op->band_n_split : 0;
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_operator_bins_info(const psi_operator* op, int32_t* block_users, int32_t* rows,
                                  int32_t* col_blocks, int32_t* bins, int32_t* split_rows,
                                  int64_t* runs) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "operator must not be NULL");
  const bool b = op->bins_built;
  if (block_users) *block_users = b ? psi::kBinsCols : 0;
  if (rows) *rows = b ? psi::kBinsRows : 0;
  if (col_blocks) *col_blocks = b ? op->bins_B : 0;
  if (bins) *bins = b ? op->bins_nb : 0;
  if (split_rows) *split_rows = b ? op->bins_n_split : 0;
  if (runs) *runs = b ? op->bins_runs : 0;
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_debug_force_slot_timeout(psi_operator* op, int32_t on) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "operator must not be NULL");
  PSI_REQUIRE(on == 0 || on == 1, "on must be 0 or 1");
  psi_status s = psi::check_device(op);
  if (s != PSI_OK) return s;
  const int v = on;
  for (int k = 0; k < 2; ++k)
    PSI_HIP_CHECK(hipMemcpy(&op->ctrl[k].force_timeout, &v, sizeof(v), hipMemcpyHostToDevice));
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_pass_time(psi_operator* op, int32_t pass_kind, int32_t reps, int32_t tile_items,
                         int32_t col_segments, int32_t seg_form, double* mean_ms,
                         void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  PSI_REQUIRE(op->n_graphs == 1, "psi_pass_time needs a single-graph operator");
  psi_status st = psi::check_device(op);
  if (st != PSI_OK) return st;
  return psi::pass_time(op, pass_kind, reps, tile_items, col_segments, seg_form, mean_ms,
                        static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_autotune(psi_operator* op, int32_t precision, int32_t reps, int32_t* tile_items,
                        int32_t* col_segments, int32_t* seg_form, double* best_ms,
                        void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status st = psi::check_device(op);
  if (st != PSI_OK) return st;
  int t = 0, sg = 0, fm = 0;
  st = psi::autotune(op, precision, reps, &t, &sg, &fm, best_ms,
                     static_cast<hipStream_t>(stream));
  if (st == PSI_OK) {
    if (tile_items) *tile_items = t;
    if (col_segments) *col_segments = sg;
    if (seg_form) *seg_form = fm;
  }
  return st;
  PSI_GUARD_END
}

psi_status psi_autotune_batched(psi_operator* op, int32_t precision, int32_t n_scenarios,
                                void* workspace, size_t workspace_bytes, int32_t reps,
                                int32_t* batch_tile, int32_t* batch_items, int32_t* hub_chunk,
                                double* best_ms, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status st = psi::check_device(op);
  if (st != PSI_OK) return st;
  int bt = 0, bi = 0, bc = 0;
  st = psi::autotune_batched(op, precision, n_scenarios, workspace, workspace_bytes, reps, &bt,
                             &bi, &bc, best_ms, static_cast<hipStream_t>(stream));
  if (st == PSI_OK) {
    if (batch_tile) *batch_tile = bt;
    if (batch_items) *batch_items = bi;
    if (hub_chunk) *hub_chunk = bc;
  }
  return st;
  PSI_GUARD_END
}

psi_status psi_autotune_graphs(psi_operator* op, int32_t precision, double tol, int32_t reps,
                               int32_t* tile_items, int32_t* col_segments, int32_t* seg_form,
                               double* best_ms, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status st = psi::check_device(op);
  if (st != PSI_OK) return st;
  int t = 0, sg = 0, fm = 0;
  st = psi::autotune_graphs(op, precision, tol, reps, &t, &sg, &fm, best_ms,
                            static_cast<hipStream_t>(stream));
  if (st == PSI_OK) {
    if (tile_items) *tile_items = t;
    if (col_segments) *col_segments = sg;
    if (seg_form) *seg_form = fm;
  }
  return st;
  PSI_GUARD_END
}

psi_status psi_batched_workspace_size(const psi_operator* op, int32_t n_scenarios,
                                      int32_t precision, size_t* bytes) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  if (op->n_graphs > 1) {
    PSI_REQUIRE(bytes, "bytes must not be NULL");
    *bytes = 0;
    return PSI_OK;
  }
  return psi::batched_workspace_size(op, n_scenarios, precision, bytes);
  PSI_GUARD_END
}

psi_status psi_solve_batched(psi_operator* op, const psi_params* prm, int32_t n_scenarios,
                             const double* lambda, const double* mu, double* psi_out,
                             psi_info* infos, void* workspace, size_t workspace_bytes,
                             void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status st = psi::check_device(op);
  if (st != PSI_OK) return st;
  if (op->n_graphs > 1) {
    PSI_REQUIRE(n_scenarios == 1 && !lambda && !mu,
                "graph mode: n_scenarios must be 1 and lambda, mu NULL");
    return psi::solve_graphs(op, prm, psi_out, infos, static_cast<hipStream_t>(stream));
  }
  return psi::solve_batched(op, prm, n_scenarios, lambda, mu, psi_out, infos, workspace,
                            workspace_bytes, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_gather_probe(const double* x, int64_t n_x, int32_t col_segments,
                            const int32_t* idx, int64_t n_idx, double* out, int32_t grid,
                            int32_t reps, double* mean_ms, void* stream) {
  PSI_GUARD_BEGIN
  return psi::gather_probe(x, n_x, col_segments, idx, n_idx, out, grid, reps, mean_ms,
                           static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_anderson_workspace_size(const psi_operator* op, int32_t depth, size_t* bytes) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  return psi::anderson_workspace_size(op, depth, bytes);
  PSI_GUARD_END
}

psi_status psi_solve_anderson_noalloc(psi_operator* op, const psi_params* prm, int32_t depth,
                                      const double* s0, double* psi_out, double* s_out,
                                      psi_info* info, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status s = psi::check_device(op);
  if (s != PSI_OK) return s;
  return psi::solve_anderson_noalloc(op, prm, depth, s0, psi_out, s_out, info,
                                     static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_solve_anderson(psi_operator* op, const psi_params* prm, int32_t depth,
                              const double* s0, double* psi_out, double* s_out, psi_info* info,
                              void* workspace, size_t workspace_bytes, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status st = psi::check_device(op);
  if (st != PSI_OK) return st;
  return psi::solve_anderson(op, prm, depth, s0, psi_out, s_out, info, workspace,
                             workspace_bytes, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_solve_origins(psi_operator* op, const psi_params* prm, int32_t n_origins,
                             const int32_t* origins, double* p_out, double* psi_out,
                             psi_info* infos, void* workspace, size_t workspace_bytes,
                             void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(op, "op must not be NULL");
  psi_status st = psi::check_device(op);
  if (st != PSI_OK) return st;
  return psi::solve_origins(op, prm, n_origins, origins, p_out, psi_out, infos, workspace,
                            workspace_bytes, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

/* ---- learned warm start ---------------------------------------------------- */
int64_t psi_mpnn_param_count(void) { return psi::mpnn_param_count(); }

psi_status psi_model_state_size(size_t* bytes) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(bytes, "bytes must not be NULL");
  *bytes = psi::model_state_size();
  return PSI_OK;
  PSI_GUARD_END
}

psi_status psi_model_create(const float* params, int64_t n_params, uint32_t flags, void* state,
                            size_t state_bytes, void* stream, psi_model** model) {
  PSI_GUARD_BEGIN
  return psi::model_create(params, n_params, flags, state, state_bytes,
                           static_cast<hipStream_t>(stream), model);
  PSI_GUARD_END
}

psi_status psi_model_destroy(psi_model* model) {
  PSI_GUARD_BEGIN
  return psi::model_destroy(model);
  PSI_GUARD_END
}

psi_status psi_model_params(const psi_model* model, float* out, uint32_t flags, void* stream) {
  PSI_GUARD_BEGIN
  return psi::model_get(model, 0, out, flags, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_model_grad(const psi_model* model, float* out, uint32_t flags, void* stream) {
  PSI_GUARD_BEGIN
  return psi::model_get(model, 1, out, flags, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_mpnn_workspace_size(const psi_operator* op, int32_t training, size_t* bytes) {
  PSI_GUARD_BEGIN
  return psi::mpnn_workspace_size(op, training, bytes);
  PSI_GUARD_END
}

psi_status psi_mpnn_forward(psi_model* model, psi_operator* op, float* t_hat, double* s0,
                            void* workspace, size_t workspace_bytes, void* stream) {
  PSI_GUARD_BEGIN
  return psi::mpnn_forward(model, op, t_hat, s0, workspace, workspace_bytes,
                           static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_warmstart(psi_model* model, psi_operator* op, double* s0_out, void* workspace,
                         size_t workspace_bytes, void* stream) {
  PSI_GUARD_BEGIN
  PSI_REQUIRE(s0_out, "s0_out must not be NULL");
  return psi::mpnn_forward(model, op, nullptr, s0_out, workspace, workspace_bytes,
                           static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_mpnn_loss_backward(psi_model* model, psi_operator* op, const double* s_target,
                                  double* loss, float* t_hat, void* workspace,
                                  size_t workspace_bytes, void* stream) {
  PSI_GUARD_BEGIN
  return psi::mpnn_loss_backward(model, op, s_target, loss, t_hat, workspace, workspace_bytes,
                                 static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

psi_status psi_mpnn_adam_step(psi_model* model, double lr, double beta1, double beta2, double eps,
                              void* stream) {
  PSI_GUARD_BEGIN
  return psi::mpnn_adam_step(model, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream));
  PSI_GUARD_END
}

}  // extern "C"
