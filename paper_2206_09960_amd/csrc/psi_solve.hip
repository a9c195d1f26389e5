// Solve drivers: Algorithm 2 (Power-ψ) on the device.
//
// The host only enqueues passes and, every few passes, reads a pinned copy of
// the device control block; the gap test of eq. (condition) is made on the
// device — for a pass of the solve loop by workgroup 0 of the next pass (or by
// a one-workgroup kernel at the end of a batch) — and passes after the one
// that met it exit at once.  The number of passes between host checks is
// predicted from the observed geometric decay of the gap.
//
// PSI_PREC_MIXED refines in FP64 around FP32 correction solves: with
// r = Aᵀs + c − s computed in FP64 (one FP64 pass, whose L1 norm is also the
// gap of eq. eps_t), the correction e = Aᵀe + r is iterated in FP32 to a
// relative tolerance and s ← s + e.  The fixed point of eq. (power_psi) is
// unchanged; only the arithmetic of the correction is FP32.
#include <cfloat>
#include <algorithm>
#include <cmath>
#include <limits>

#include "psi_internal.h"

namespace psi {

bool tile_items_supported(int t);

namespace {

inline unsigned grid_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

__global__ void k_init64(const double* s0, const double* c, const double* invden, int64_t n,
                         double* s, double* z) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = s0 ? s0[i] : c[i];
  s[i] = v;
  z[i] = invden[i] * v;
}

__global__ void k_init32(const double* s0, const double* c, const float* invden32, int64_t n,
                         float* e, float* ze) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = static_cast<float>(s0 ? s0[i] : c[i]);
  e[i] = v;
  ze[i] = invden32[i] * v;
}

__global__ void k_ctrl_set(Ctrl* c, double tol, int tol_mode, int max_iter, double bnorm) {
  c->ticket = 0;
  c->done = 0;
  c->done_pass = -1;
  c->pending = 0;
  c->iter = 0;
  c->status = 0;
  c->gap = 0.0;
  c->l1 = 0.0;
  c->snorm = 0.0;
  c->tol = tol;
  c->tol_mode = tol_mode;
  c->max_iter = max_iter;
  c->bnorm = bnorm;
}

// The FP32 correction solve e = Aᵀe + r stops at eta·‖r‖₁, or at half the outer
// tolerance (in L1 units) when that is larger: after the correction the
// outer residual is about the correction's last step, so solving it below
// the outer tolerance buys nothing (the last refinement would otherwise run
// several passes past what the outer test needs).
__global__ void k_ctrl_inner(const Ctrl* outer, Ctrl* inner, double eta, int max_iter) {
  double target = outer->tol;  // the outer test in L1 units
  if (outer->tol_mode == PSI_TOL_BNORM) target = outer->bnorm > 0.0 ? outer->tol / outer->bnorm : 0.0;
  else if (outer->tol_mode == PSI_TOL_REL_L1) target = outer->tol * outer->snorm;
  inner->ticket = 0;
  inner->done = 0;
  inner->done_pass = -1;
  inner->pending = 0;
  inner->iter = 0;
  inner->status = 0;
  inner->gap = 0.0;
  inner->l1 = 0.0;
  inner->tol = fmax(eta * outer->l1, 0.5 * target);
  inner->tol_mode = PSI_TOL_ABS_L1;
  inner->max_iter = max_iter;
  inner->bnorm = 1.0;
}

// r = s_new − s_old (the FP64 residual Aᵀs + c − s), rounded to FP32; e_0 = r.
__global__ void k_prep_inner(const double* s_new, const double* s_old, const float* invden32,
                             int64_t n, float* r32, float* e, float* ze) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float r = static_cast<float>(s_new[i] - s_old[i]);
  r32[i] = r;
  e[i] = r;
  ze[i] = invden32[i] * r;
}

__global__ void k_update(double* s, const float* e, const double* invden, int64_t n, double* z) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = s[i] + static_cast<double>(e[i]);
  s[i] = v;
  z[i] = invden[i] * v;
}

__global__ void k_e_to_s(const float* e, const double* invden, int64_t n, double* s, double* z) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = static_cast<double>(e[i]);
  s[i] = v;
  z[i] = invden[i] * v;
}

__global__ void k_make_z(const double* s, const double* invden, int64_t n, double* z) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) z[i] = invden[i] * s[i];
}

__global__ void k_fill_slots(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u32(unsigned* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

__global__ void k_ctrl_clear_wait(Ctrl* c) {
  for (int k = 0; k < 2; ++k) {
    c[k].ticket = 0;
    c[k].pending = 0;
    c[k].err_flags &= ~static_cast<unsigned>(kErrSlotTimeout);
  }
}

struct IterResult {
  int iters = 0;       // passes that ran on the device (ctrl->iter)
  int status = PSI_OK;
  double gap = 0.0;
  double l1 = 0.0;
  bool stagnated = false;
};

// Column segments for a gathered vector of `bytes` per user: enough that one
// segment (the share of an XCD group) stays near half of a 4 MB L2.
int auto_segments(const psi_operator* op, int bytes) {
  const double xb = static_cast<double>(op->n) * bytes;
  if (xb <= 3.0e6) return 1;
  int S = 2;
  while (S < 8 && xb / S > 2.5e6) S *= 2;
  return S;
}

psi_status resolve_segments(const psi_operator* op, int requested, int bytes, int* S) {
  PSI_REQUIRE(requested == 0 || requested == 1 || requested == 2 || requested == 4 ||
                  requested == 8,
              "col_segments must be 0, 1, 2, 4 or 8");
  *S = requested ? requested : auto_segments(op, bytes);
  return PSI_OK;
}

// Enqueue passes until the device sets done; make(i) gives the arguments of
// pass i (i counts passes enqueued in this call).
template <class Make>
psi_status iterate(psi_operator* op, int S, int ctrl_idx, PassMode mode, Make make, int max_iter,
                   int check_every, hipStream_t st, IterResult* out) {
  Ctrl* dctrl = op->ctrl + ctrl_idx;
  Ctrl* hctrl = op->host_ctrl + ctrl_idx;
  int enq = 0;
  int k = check_every > 0 ? check_every : 6;
  double prev_gap = -1.0;
  int prev_iter = 0;
  double best = std::numeric_limits<double>::infinity();
  int best_iter = 0;
  while (true) {
    const int cnt = std::min(k, max_iter - enq);
    // deferred gaps: pass p stores its per-workgroup pairs in buffer p mod 2
    // and the next pass's workgroup 0 decides on them, so no pass ends with
    // a chain of reductions; the batch's last pairs are decided before the
    // host reads the control block
    for (int i = 0; i < cnt; ++i) {
      const int p = enq + i;
      PassArgs a = make(p);
      a.defer_gap = 1;
      a.pass_id = p;
      a.gap_part = op->gap_part + size_t(p & 1) * 2 * kMaxGrid;
      a.gap_prev = op->gap_part + size_t((p & 1) ^ 1) * 2 * kMaxGrid;
      psi_status s = run_pass(op, S, mode, a, st);
      if (s != PSI_OK) return s;
    }
    enq += cnt;
    {
      psi_status s = launch_gap_decide(dctrl, op->gap_part + size_t((enq - 1) & 1) * 2 * kMaxGrid,
                                       op->hist, 1, st);
      if (s != PSI_OK) return s;
    }
    PSI_HIP_CHECK(hipMemcpyAsync(hctrl, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    if (hctrl->err_flags & kErrSlotTimeout) return check_waits(op, st);  // never expected
    out->iters = hctrl->iter;
    out->gap = hctrl->gap;
    out->l1 = hctrl->l1;
    out->status = hctrl->status;
    if (hctrl->done) return PSI_OK;
    if (enq >= max_iter) {
      out->status = PSI_ENOTCONV;
      return PSI_OK;
    }
    const double gap = hctrl->gap;
    const int it = hctrl->iter;
    if (gap < best * (1.0 - 1e-3)) {
      best = gap;
      best_iter = it;
    } else if (it - best_iter >= 25) {
      out->status = PSI_ESTAGNATED;
      out->stagnated = true;
      return PSI_OK;
    }
    if (check_every == 0) {
      if (prev_gap > 0.0 && gap > 0.0 && gap < prev_gap && it > prev_iter) {
        const double rate = std::pow(gap / prev_gap, 1.0 / (it - prev_iter));
        const double need = std::log(hctrl->tol / gap) / std::log(rate);
        k = static_cast<int>(std::clamp(std::ceil(need), 1.0, 64.0));
      } else {
        k = std::min(2 * k, 64);
      }
      prev_gap = gap;
      prev_iter = it;
    }
  }
}

}  // namespace

psi_status mixed_inner_begin(psi_operator* op, const double* Y, const double* X, double eta,
                             int max_iter, hipStream_t st) {
  const int64_t n = op->n;
  hipLaunchKernelGGL(k_prep_inner, dim3(grid_for(n)), dim3(kBlock), 0, st, Y, X, op->invden32, n,
                     op->r32, op->e_a, op->ze_a);
  hipLaunchKernelGGL(k_ctrl_inner, dim3(1), dim3(1), 0, st, op->ctrl, op->ctrl + 1, eta,
                     max_iter);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

psi_status mixed_update(psi_operator* op, double* X, const float* e, double* zX, hipStream_t st) {
  const int64_t n = op->n;
  hipLaunchKernelGGL(k_update, dim3(grid_for(n)), dim3(kBlock), 0, st, X, e, op->invden, n, zX);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

psi_status check_waits(psi_operator* op, hipStream_t st) {
  Ctrl* h = op->host_ctrl;
  PSI_HIP_CHECK(hipMemcpyAsync(h, op->ctrl, 2 * sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  if (!((h[0].err_flags | h[1].err_flags) & kErrSlotTimeout)) return PSI_OK;
  // a partial that arrives after its reader gave up must not be read by a
  // later pass: empty every slot and ticket again
  auto fill = [&](void* p, int64_t cnt) {
    if (p && cnt > 0)
      hipLaunchKernelGGL(k_fill_slots, dim3(unsigned(std::min<int64_t>(1024, (cnt + 255) / 256))),
                         dim3(256), 0, st, static_cast<unsigned long long*>(p), cnt, kEmptySlot);
  };
  auto zero = [&](unsigned* p, int64_t cnt) {
    if (p && cnt > 0)
      hipLaunchKernelGGL(k_fill_u32, dim3(unsigned(std::min<int64_t>(1024, (cnt + 255) / 256))),
                         dim3(256), 0, st, p, cnt);
  };
  fill(op->part_open, op->max_tiles);
  fill(op->seg_part_open, op->max_seg_tiles);
  fill(op->slice_part, op->cap_chunks);
  zero(op->slice_ticket, op->cap_chunks);
  fill(op->gap_part, 4 * int64_t(kMaxGrid));
  fill(op->gap_grp, 2 * int64_t(kMaxGrid / 64));
  zero(op->grp_ticket, kMaxGrid / 64);
  hipLaunchKernelGGL(k_ctrl_clear_wait, dim3(1), dim3(1), 0, st, op->ctrl);
  PSI_HIP_CHECK(hipGetLastError());
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  set_error("a bounded wait for a partial of another workgroup gave up: the result of this "
            "call is invalid (the operator's slots were emptied, later calls are unaffected)");
  return PSI_EDEVICE;
}

// Layout of a call's passes.  The band layout when it is requested, or when
// nothing is requested (seg_form = col_segments = 0) and it was tuned for this
// precision or, untuned, the gathered vector (`bytes` per user) exceeds
// kBandAutoBytes on a single-graph operator.  Otherwise the partial-pass form
// for S segments: the requested one, else the tuned one (when it was tuned for
// this S), else sliced while a segment's share of the gathered vector is at
// most 6 MB, about what an XCD's L2 keeps.
constexpr double kBandAutoBytes = 32.0e6;

psi_status resolve_form(const psi_operator* op, int requested, int requested_S, int precision,
                        int S, int bytes, int* form) {
  PSI_REQUIRE(requested == 0 || requested == PSI_SEG_TILES || requested == PSI_SEG_SLICES ||
                  requested == PSI_SEG_BANDS || requested == PSI_SEG_BINS,
              "seg_form must be 0, PSI_SEG_TILES, PSI_SEG_SLICES, PSI_SEG_BANDS or PSI_SEG_BINS");
  const bool untuned = op->tuned_tile[precision] == 0;
  if (requested == kSegBins ||
      (requested == 0 && requested_S == 0 && precision != PSI_PREC_FP64_WEIGHTED &&
       op->n_graphs == 1 && op->tuned_form[precision] == kSegBins)) {
    PSI_REQUIRE(op->n_graphs == 1, "the binned layout is for single-graph operators");
    PSI_REQUIRE(precision != PSI_PREC_FP64_WEIGHTED, "the weighted pass has no binned layout");
    *form = kSegBins;
  } else if (requested == kSegBands ||
      (requested == 0 && requested_S == 0 && precision != PSI_PREC_FP64_WEIGHTED &&
       op->n_graphs == 1 &&
       (op->tuned_form[precision] == kSegBands ||
        (untuned && static_cast<double>(op->n) * bytes >= kBandAutoBytes)))) {
    PSI_REQUIRE(op->n_graphs == 1, "the band layout is for single-graph operators");
    PSI_REQUIRE(precision != PSI_PREC_FP64_WEIGHTED, "the weighted pass has no band layout");
    *form = kSegBands;
  } else if (S <= 1) {
    *form = 0;
  } else if (requested) {
    *form = requested;
  } else if (op->tuned_form[precision] && op->tuned_S[precision] == S) {
    *form = op->tuned_form[precision];
  } else {
    *form = static_cast<double>(op->n) * bytes / S <= 6.0e6 ? kSegSlices : kSegTiles;
  }
  return PSI_OK;
}

// Tuned for `precision`, else the layout already built, else 2^18 x 2048.
void band_params(const psi_operator* op, int precision, int* wlog, int* rows) {
  if (op->tuned_band_wlog[precision]) {
    *wlog = op->tuned_band_wlog[precision];
    *rows = op->tuned_band_rows[precision];
  } else if (op->band_built) {
    *wlog = op->band_wlog;
    *rows = op->band_rows;
  } else {
    *wlog = kBandMaxLog;
    *rows = 2048;
  }
}

// Schedules and layouts the passes of one call need; the passes of the call
// then use `form` (band layout with column blocks of 2^wlog users and row
// blocks of `rows` rows; 0 = those of op->band_* if built, else the defaults).
psi_status prepare(psi_operator* op, int tile, int S, int form, hipStream_t st, int wlog,
                   int rows) {
  psi_status s = ensure_schedule(op, tile, st);
  if (s != PSI_OK) return s;
  op->seg_form = 0;
  if (form == kSegBins) {
    s = ensure_bins(op, st);
    if (s != PSI_OK) return s;
    op->seg_form = kSegBins;
    return PSI_OK;
  }
  if (form == kSegBands) {
    if (!wlog) wlog = op->band_built ? op->band_wlog : kBandMaxLog;
    if (!rows) rows = op->band_built ? op->band_rows : 2048;
    s = ensure_bands(op, wlog, rows, st);
    if (s != PSI_OK) return s;
    op->seg_form = kSegBands;
    return PSI_OK;
  }
  if (S <= 1) return PSI_OK;
  s = ensure_segments(op, S, st);
  if (s != PSI_OK) return s;
  s = form == kSegSlices ? ensure_seg_slices(op, st) : ensure_seg_tiles(op, tile, st);
  if (s != PSI_OK) return s;
  op->seg_form = form;
  return PSI_OK;
}

psi_status prepare(psi_operator* op, int tile, int S, int form, hipStream_t st) {
  return prepare(op, tile, S, form, st, 0, 0);
}

// prepare() with the band parameters tuned for `precision` (or the defaults).
psi_status prepare_for(psi_operator* op, int precision, int tile, int S, int form,
                       hipStream_t st, int wlog = 0, int rows = 0) {
  PSI_REQUIRE(wlog == 0 || (wlog >= kBandMinLog && wlog <= kBandMaxLog),
              "band_col_log must be 0, 17 or 18");
  PSI_REQUIRE(rows == 0 || band_rows_supported(rows),
              "band_rows must be 0, 1024, 1280, 1536 or 2048");
  if (form == kSegBands) {
    int tw = 0, tr = 0;
    band_params(op, precision, &tw, &tr);
    if (!wlog) wlog = tw;
    if (!rows) rows = tr;
  }
  psi_status s = prepare(op, tile, S, form, st, wlog, rows);
  if (s != PSI_OK) return s;
  // the pacing tuned for this layout, else none
  op->band_pace_ticks = form == kSegBands && op->tuned_band_wlog[precision] == wlog &&
                                op->tuned_band_rows[precision] == rows
                            ? op->tuned_band_pace[precision]
                            : 0ull;
  return PSI_OK;
}

psi_status solve(psi_operator* op, const psi_params* prm, const double* s0, double* psi_out,
                 double* s_out, psi_info* info, hipStream_t st) {
  PSI_REQUIRE(prm, "params must not be NULL");
  PSI_REQUIRE(psi_out, "psi_out must not be NULL");
  PSI_REQUIRE(prm->tol > 0.0 && std::isfinite(prm->tol), "tol must be finite and > 0");
  PSI_REQUIRE(prm->max_iter > 0, "max_iter must be > 0");
  PSI_REQUIRE(prm->tol_mode >= PSI_TOL_ABS_L1 && prm->tol_mode <= PSI_TOL_REL_L1,
              "unknown tol_mode");
  PSI_REQUIRE(prm->precision >= PSI_PREC_FP64 && prm->precision <= PSI_PREC_FP32,
              "unknown precision");
  PSI_REQUIRE(prm->check_every >= 0, "check_every must be >= 0");
  PSI_REQUIRE(prm->precision != PSI_PREC_FP64_WEIGHTED || op->val64,
              "PSI_PREC_FP64_WEIGHTED needs an operator built with PSI_WEIGHTED_FP64");
  PSI_REQUIRE(op->n_graphs == 1, "multi-graph operators are solved by psi_solve_batched");
  const int tuned_tile = op->tuned_tile[prm->precision];
  const int tile = prm->tile_items ? prm->tile_items
                 : tuned_tile      ? tuned_tile
                 : (op->sched_items ? op->sched_items : kDefaultTileItems);
  PSI_REQUIRE(tile_items_supported(tile), "unsupported tile_items");
  int S = 1;
  const int want_S = prm->col_segments ? prm->col_segments : op->tuned_S[prm->precision];
  psi_status s = resolve_segments(op, want_S, prm->precision == PSI_PREC_FP64 ? 8 : 4, &S);
  if (s != PSI_OK) return s;
  if (prm->precision == PSI_PREC_FP64_WEIGHTED) S = 1;
  int form = 0;
  s = resolve_form(op, prm->seg_form, prm->col_segments, prm->precision, S,
                   prm->precision == PSI_PREC_FP64 ? 8 : 4, &form);
  if (s != PSI_OK) return s;
  if (form == kSegBands || form == kSegBins) S = 1;
  s = prepare_for(op, prm->precision, tile, S, form, st, prm->band_col_log, prm->band_rows);
  if (s != PSI_OK) return s;

  const int64_t n = op->n;
  const double bnorm = op->stats.b_norm;
  const double kap = op->stats.kappa;
  EventPair tm;
  PSI_HIP_CHECK(hipEventCreate(&tm.a));
  PSI_HIP_CHECK(hipEventCreate(&tm.b));
  PSI_HIP_CHECK(hipEventRecord(tm.a, st));

  PassArgs base = base_args(op);
  psi_info inf{};
  inf.b_norm = bnorm;
  inf.kappa = kap;
  inf.used_s0 = s0 ? 1 : 0;
  inf.col_segments = S;
  inf.tile_items = tile;
  inf.seg_form = form;

  // optional start: keep s0 only if its fixed-point residual beats c's.
  // ‖r(c)‖₁ depends only on the operator and is computed once.  In FP64 the
  // pass from s0 is the solve's first iteration (counted, with its gap test),
  // and the iteration continues from its output when s0 is kept.
  bool s0_stepped = false;
  if (s0 && !(prm->flags & PSI_NO_FALLBACK)) {
    if (!(op->rc_l1 >= 0.0)) {
      hipLaunchKernelGGL(k_init64, dim3(grid_for(n)), dim3(kBlock), 0, st, nullptr, op->c,
                         op->invden, n, op->s_a, op->z_a);
      PassArgs a = base;
      a.x = op->z_a;
      a.s_old = op->s_a;
      a.s_new = op->s_b;
      a.z_new = op->z_b;
      a.gap_out = op->scal;
      a.count_iter = 0;
      a.respect_done = 0;
      a.ctrl = op->ctrl + 1;
      s = run_pass(op, S, kStep64, a, st);
      if (s != PSI_OK) return s;
      inf.spmv_passes += 1;
      double rc = 0.0;
      PSI_HIP_CHECK(hipMemcpyAsync(&rc, op->scal, sizeof(rc), hipMemcpyDeviceToHost, st));
      s = check_waits(op, st);
      if (s != PSI_OK) return s;
      op->rc_l1 = rc;
    }
    const bool first_iter = prm->precision == PSI_PREC_FP64;
    hipLaunchKernelGGL(k_init64, dim3(grid_for(n)), dim3(kBlock), 0, st, s0, op->c, op->invden,
                       n, op->s_a, op->z_a);
    if (first_iter)
      hipLaunchKernelGGL(k_ctrl_set, dim3(1), dim3(1), 0, st, op->ctrl, prm->tol, prm->tol_mode,
                         prm->max_iter, bnorm);
    PassArgs a = base;
    a.x = op->z_a;
    a.s_old = op->s_a;
    a.s_new = op->s_b;
    a.z_new = op->z_b;
    a.gap_out = op->scal + 1;
    a.count_iter = first_iter ? 1 : 0;
    a.respect_done = 0;
    a.ctrl = first_iter ? op->ctrl : op->ctrl + 1;
    s = run_pass(op, S, kStep64, a, st);
    if (s != PSI_OK) return s;
    double r1 = 0.0;
    PSI_HIP_CHECK(hipMemcpyAsync(&r1, op->scal + 1, sizeof(r1), hipMemcpyDeviceToHost, st));
    s = check_waits(op, st);
    if (s != PSI_OK) return s;
    if (!(r1 <= op->rc_l1)) {  // c wins: the step from s0 is discarded
      s0 = nullptr;
      inf.used_s0 = 0;
      inf.spmv_passes += 1;
    } else if (first_iter) {
      s0_stepped = true;  // the step is the solve's first iteration, counted below
    } else {
      inf.spmv_passes += 1;
    }
  }

  double* s_fin = nullptr;
  double* z_fin = nullptr;
  int status = PSI_OK;
  double last_l1 = 0.0;
  const int prec = prm->precision;

  auto plain64 = [&](double* sa, double* za, double* sb, double* zb, int max_iter,
                     IterResult* res) -> psi_status {
    const PassMode mode = prec == PSI_PREC_FP64_WEIGHTED ? kStep64W : kStep64;
    auto make = [&](int i) {
      PassArgs a = base;
      const bool even = (i & 1) == 0;
      a.x = mode == kStep64W ? static_cast<const void*>(even ? sa : sb)
                             : static_cast<const void*>(even ? za : zb);
      a.s_old = even ? sa : sb;
      a.s_new = even ? sb : sa;
      a.z_new = even ? zb : za;
      a.count_iter = 1;
      a.respect_done = 1;
      a.ctrl = op->ctrl;
      return a;
    };
    return iterate(op, S, 0, mode, make, max_iter, prm->check_every, st, res);
  };

  if (prec == PSI_PREC_FP64 || prec == PSI_PREC_FP64_WEIGHTED) {
    IterResult res;
    if (s0_stepped) {
      // (s_b, z_b) = the first step from s0, already counted by the control block;
      // pass i writes s_a for even i, so iteration t ends in s_b when t is odd
      s = plain64(op->s_b, op->z_b, op->s_a, op->z_a, prm->max_iter - 1, &res);
    } else {
      hipLaunchKernelGGL(k_init64, dim3(grid_for(n)), dim3(kBlock), 0, st, s0, op->c,
                         op->invden, n, op->s_a, op->z_a);
      hipLaunchKernelGGL(k_ctrl_set, dim3(1), dim3(1), 0, st, op->ctrl, prm->tol,
                         prm->tol_mode, prm->max_iter, bnorm);
      s = plain64(op->s_a, op->z_a, op->s_b, op->z_b, prm->max_iter, &res);
    }
    if (s != PSI_OK) return s;
    inf.iterations = res.iters;
    inf.spmv_passes += res.iters;
    status = res.status;
    inf.final_gap = res.gap;
    last_l1 = res.l1;
    const bool odd = res.iters & 1;
    s_fin = odd ? op->s_b : op->s_a;
    z_fin = odd ? op->z_b : op->z_a;
    if (prec == PSI_PREC_FP64_WEIGHTED) {
      hipLaunchKernelGGL(k_make_z, dim3(grid_for(n)), dim3(kBlock), 0, st, s_fin, op->invden, n,
                         z_fin);
    }
  } else if (prec == PSI_PREC_FP32) {
    hipLaunchKernelGGL(k_init32, dim3(grid_for(n)), dim3(kBlock), 0, st, s0, op->c, op->invden32,
                       n, op->e_a, op->ze_a);
    hipLaunchKernelGGL(k_ctrl_set, dim3(1), dim3(1), 0, st, op->ctrl, prm->tol, prm->tol_mode,
                       prm->max_iter, bnorm);
    auto make = [&](int i) {
      PassArgs a = base;
      const bool even = (i & 1) == 0;
      a.x = even ? op->ze_a : op->ze_b;
      a.r32 = op->c32;
      a.e_old = even ? op->e_a : op->e_b;
      a.e_new = even ? op->e_b : op->e_a;
      a.ze_new = even ? op->ze_b : op->ze_a;
      a.count_iter = 1;
      a.respect_done = 1;
      a.ctrl = op->ctrl;
      return a;
    };
    IterResult res;
    s = iterate(op, S, 0, kStep32, make, prm->max_iter, prm->check_every, st, &res);
    if (s != PSI_OK) return s;
    inf.iterations = res.iters;
    inf.fp32_passes = res.iters;
    inf.spmv_passes += res.iters;
    status = res.status;
    inf.final_gap = res.gap;
    last_l1 = res.l1;
    const float* e_fin = (res.iters & 1) ? op->e_b : op->e_a;
    hipLaunchKernelGGL(k_e_to_s, dim3(grid_for(n)), dim3(kBlock), 0, st, e_fin, op->invden, n,
                       op->s_a, op->z_a);
    s_fin = op->s_a;
    z_fin = op->z_a;
  } else {  // PSI_PREC_MIXED
    const double eta = prm->inner_tol > 0.0 ? prm->inner_tol : 2e-6;
    double* X = op->s_a;
    double* zX = op->z_a;
    double* Y = op->s_b;
    double* zY = op->z_b;
    hipLaunchKernelGGL(k_init64, dim3(grid_for(n)), dim3(kBlock), 0, st, s0, op->c, op->invden,
                       n, X, zX);
    hipLaunchKernelGGL(k_ctrl_set, dim3(1), dim3(1), 0, st, op->ctrl, prm->tol, prm->tol_mode,
                       prm->max_iter, bnorm);
    double prev_gap = std::numeric_limits<double>::infinity();
    int fp64_passes = 0;
    bool finished = false;
    while (!finished) {
      // FP64 residual pass: Y = Aᵀ X + c, gap = ‖Y − X‖₁ (tol_mode units)
      PassArgs a = base;
      a.x = zX;
      a.s_old = X;
      a.s_new = Y;
      a.z_new = zY;
      a.count_iter = 1;
      a.respect_done = 0;
      a.ctrl = op->ctrl;
      s = run_pass(op, S, kStep64, a, st);
      if (s != PSI_OK) return s;
      ++fp64_passes;
      Ctrl* h = op->host_ctrl;
      s = check_waits(op, st);  // copies both control blocks to the host
      if (s != PSI_OK) return s;
      inf.final_gap = h->gap;
      last_l1 = h->l1;
      s_fin = Y;
      z_fin = zY;
      if (h->done) {
        status = h->status;
        break;
      }
      if (!(h->gap < 0.25 * prev_gap)) {
        // refinement no longer gains: finish with plain FP64 steps from Y
        const int before = h->iter;
        IterResult res;
        s = plain64(Y, zY, X, zX, prm->max_iter - fp64_passes, &res);
        if (s != PSI_OK) return s;
        fp64_passes = res.iters;  // ctrl->iter kept counting from the refinement passes
        status = res.status;
        inf.final_gap = res.gap;
        last_l1 = res.l1;
        const int extra = res.iters - before;
        const bool odd = extra & 1;
        s_fin = odd ? X : Y;
        z_fin = odd ? zX : zY;
        break;
      }
      prev_gap = h->gap;
      // FP32 correction solve e = Aᵀe + r
      s = mixed_inner_begin(op, Y, X, eta, prm->max_iter, st);
      if (s != PSI_OK) return s;
      auto make = [&](int i) {
        PassArgs b = base;
        const bool even = (i & 1) == 0;
        b.x = even ? op->ze_a : op->ze_b;
        b.r32 = op->r32;
        b.e_old = even ? op->e_a : op->e_b;
        b.e_new = even ? op->e_b : op->e_a;
        b.ze_new = even ? op->ze_b : op->ze_a;
        b.count_iter = 1;
        b.respect_done = 1;
        b.ctrl = op->ctrl + 1;
        return b;
      };
      IterResult res;
      s = iterate(op, S, 1, kStep32, make, prm->max_iter, prm->check_every, st, &res);
      if (s != PSI_OK) return s;
      inf.fp32_passes += res.iters;
      if (res.status == PSI_ENUMERIC) {
        status = PSI_ENUMERIC;
        break;
      }
      const float* e_fin = (res.iters & 1) ? op->e_b : op->e_a;
      s = mixed_update(op, X, e_fin, zX, st);
      if (s != PSI_OK) return s;
      inf.refinements += 1;
      if (fp64_passes >= prm->max_iter) {
        status = PSI_ENOTCONV;
        break;
      }
    }
    inf.iterations = fp64_passes;
    inf.spmv_passes += fp64_passes + inf.fp32_passes;
  }

  // ψ = (Bᵀs + d)/N from the final s (the last line of Algorithm 2)
  {
    PassArgs a = base;
    a.x = z_fin;
    a.s_new = psi_out;
    a.count_iter = 0;
    a.respect_done = 0;
    s = run_pass(op, S, kFinal64, a, st);
    if (s != PSI_OK) return s;
    inf.spmv_passes += 1;
  }
  if (s_out) PSI_HIP_CHECK(hipMemcpyAsync(s_out, s_fin, 8 * size_t(n), hipMemcpyDeviceToDevice, st));
  PSI_HIP_CHECK(hipEventRecord(tm.b, st));
  PSI_HIP_CHECK(hipEventSynchronize(tm.b));
  float ms = 0.f;
  PSI_HIP_CHECK(hipEventElapsedTime(&ms, tm.a, tm.b));
  s = check_waits(op, st);  // the final pass, like every pass, must have had all its partials
  if (s != PSI_OK) return s;
  inf.device_ms = ms;
  inf.final_l1_step = last_l1;
  inf.err_bound_s = kap < 1.0 ? kap / (1.0 - kap) * last_l1 : std::numeric_limits<double>::infinity();
  inf.psi_gap_bound = n > 0 ? last_l1 * bnorm / static_cast<double>(n) : 0.0;
  inf.status = status;
  if (info) *info = inf;
  if (status == PSI_ENOTCONV) set_error("max_iter reached before the gap fell to tol");
  else if (status == PSI_ESTAGNATED) set_error("the gap stopped decreasing above tol");
  else if (status == PSI_ENUMERIC) set_error("NaN or Inf in the iteration");
  return static_cast<psi_status>(status);
}

// Asynchronous local updates in a fixed order: block Gauss–Seidel sweeps of
// s ← Aᵀs + c over the band layout.  The bands of a sweep run one after
// another and each gathers the users of earlier bands from this sweep's new
// values (split rows are finished after the band holding their last piece), so
// later users update from fresher values, as in the local-update methods the
// paper names as follow-ups (Sec. I).  The fixed point is that of
// eq. (power_psi); the stopping test is eq. (condition) on the sweep's change
// ‖s_sweep − s_prev‖₁ in tol_mode units; ψ = (Bᵀs + d)/N from the final s.
psi_status solve_async(psi_operator* op, const psi_params* prm, const double* s0,
                       double* psi_out, double* s_out, psi_info* info, hipStream_t st) {
  PSI_REQUIRE(prm, "params must not be NULL");
  PSI_REQUIRE(psi_out, "psi_out must not be NULL");
  PSI_REQUIRE(prm->tol > 0.0 && std::isfinite(prm->tol), "tol must be finite and > 0");
  PSI_REQUIRE(prm->max_iter > 0, "max_iter must be > 0");
  PSI_REQUIRE(prm->tol_mode >= PSI_TOL_ABS_L1 && prm->tol_mode <= PSI_TOL_REL_L1,
              "unknown tol_mode");
  PSI_REQUIRE(prm->precision == PSI_PREC_FP64, "asynchronous sweeps run in PSI_PREC_FP64");
  PSI_REQUIRE(prm->check_every >= 0, "check_every must be >= 0");
  PSI_REQUIRE(op->n_graphs == 1, "asynchronous sweeps need a single-graph operator");
  PSI_REQUIRE(prm->seg_form == 0 || prm->seg_form == PSI_SEG_BANDS,
              "asynchronous sweeps run in the band layout (seg_form 0 or PSI_SEG_BANDS)");
  const int tile = op->sched_items ? op->sched_items : kDefaultTileItems;
  psi_status s = prepare_for(op, PSI_PREC_FP64, tile, 1, kSegBands, st, prm->band_col_log,
                             prm->band_rows);
  if (s != PSI_OK) return s;
  const int64_t n = op->n;
  EventPair tm;
  PSI_HIP_CHECK(hipEventCreate(&tm.a));
  PSI_HIP_CHECK(hipEventCreate(&tm.b));
  PSI_HIP_CHECK(hipEventRecord(tm.a, st));
  PassArgs base = base_args(op);
  hipLaunchKernelGGL(k_init64, dim3(grid_for(n)), dim3(kBlock), 0, st, s0, op->c, op->invden, n,
                     op->s_a, op->z_a);
  hipLaunchKernelGGL(k_ctrl_set, dim3(1), dim3(1), 0, st, op->ctrl, prm->tol, prm->tol_mode,
                     prm->max_iter, op->stats.b_norm);
  auto make = [&](int i) {
    PassArgs a = base;
    const bool even = (i & 1) == 0;
    a.x = even ? op->z_a : op->z_b;
    a.s_old = even ? op->s_a : op->s_b;
    a.s_new = even ? op->s_b : op->s_a;
    a.z_new = even ? op->z_b : op->z_a;
    a.count_iter = 1;
    a.respect_done = 1;
    a.gs_sweep = 1;
    a.ctrl = op->ctrl;
    return a;
  };
  IterResult res;
  s = iterate(op, 1, 0, kStep64, make, prm->max_iter, prm->check_every, st, &res);
  if (s != PSI_OK) return s;
  const bool odd = res.iters & 1;
  double* s_fin = odd ? op->s_b : op->s_a;
  double* z_fin = odd ? op->z_b : op->z_a;
  {
    PassArgs a = base;
    a.x = z_fin;
    a.s_new = psi_out;
    a.count_iter = 0;
    a.respect_done = 0;
    s = run_pass(op, 1, kFinal64, a, st);
    if (s != PSI_OK) return s;
  }
  if (s_out) PSI_HIP_CHECK(hipMemcpyAsync(s_out, s_fin, 8 * size_t(n), hipMemcpyDeviceToDevice, st));
  PSI_HIP_CHECK(hipEventRecord(tm.b, st));
  PSI_HIP_CHECK(hipEventSynchronize(tm.b));
  float ms = 0.f;
  PSI_HIP_CHECK(hipEventElapsedTime(&ms, tm.a, tm.b));
  s = check_waits(op, st);
  if (s != PSI_OK) return s;
  const double kap = op->stats.kappa;
  psi_info inf{};
  inf.status = res.status;
  inf.iterations = res.iters;
  inf.spmv_passes = res.iters + 1;
  inf.used_s0 = s0 ? 1 : 0;
  inf.col_segments = 1;
  inf.tile_items = tile;
  inf.seg_form = kSegBands;
  inf.final_gap = res.gap;
  inf.final_l1_step = res.l1;
  inf.b_norm = op->stats.b_norm;
  inf.kappa = kap;
  inf.err_bound_s = kap < 1.0 ? kap / (1.0 - kap) * res.l1 : std::numeric_limits<double>::infinity();
  inf.psi_gap_bound = n > 0 ? res.l1 * op->stats.b_norm / static_cast<double>(n) : 0.0;
  inf.device_ms = ms;
  if (info) *info = inf;
  if (res.status == PSI_ENOTCONV) set_error("max_iter reached before the gap fell to tol");
  else if (res.status == PSI_ESTAGNATED) set_error("the gap stopped decreasing above tol");
  else if (res.status == PSI_ENUMERIC) set_error("NaN or Inf in the iteration");
  return static_cast<psi_status>(res.status);
}

psi_status step(psi_operator* op, int precision, const double* s_in, double* s_out,
                double* gap_out, int tile_items, int col_segments, int seg_form,
                hipStream_t st) {
  PSI_REQUIRE(s_in && s_out && s_in != s_out, "s_in and s_out must be distinct device arrays");
  PSI_REQUIRE(precision == PSI_PREC_FP64 || precision == PSI_PREC_FP64_WEIGHTED,
              "psi_step supports PSI_PREC_FP64 and PSI_PREC_FP64_WEIGHTED");
  PSI_REQUIRE(precision != PSI_PREC_FP64_WEIGHTED || op->val64,
              "weighted step needs an operator built with PSI_WEIGHTED_FP64");
  const int tile = tile_items ? tile_items : (op->sched_items ? op->sched_items : kDefaultTileItems);
  PSI_REQUIRE(tile_items_supported(tile), "unsupported tile_items");
  int S = 1;
  psi_status s = resolve_segments(op, col_segments, 8, &S);
  if (s != PSI_OK) return s;
  if (precision == PSI_PREC_FP64_WEIGHTED) S = 1;
  int form = 0;
  s = resolve_form(op, seg_form, col_segments, precision, S, 8, &form);
  if (s != PSI_OK) return s;
  if (form == kSegBands || form == kSegBins) S = 1;
  s = prepare_for(op, precision, tile, S, form, st);
  if (s != PSI_OK) return s;
  PassArgs a = base_args(op);
  a.s_old = s_in;
  a.s_new = s_out;
  a.z_new = op->z_b;
  a.gap_out = gap_out;
  a.count_iter = 0;
  a.respect_done = 0;
  a.ctrl = op->ctrl + 1;
  if (precision == PSI_PREC_FP64) {
    hipLaunchKernelGGL(k_make_z, dim3(grid_for(op->n)), dim3(kBlock), 0, st, s_in, op->invden,
                       op->n, op->z_a);
    a.x = op->z_a;
    return run_pass(op, S, kStep64, a, st);
  }
  a.x = s_in;
  return run_pass(op, 1, kStep64W, a, st);
}

psi_status final_psi(psi_operator* op, const double* s_vec, double* psi_out, hipStream_t st) {
  PSI_REQUIRE(s_vec && psi_out, "s and psi_out must not be NULL");
  int S = auto_segments(op, 8);
  int form = 0;
  psi_status s = resolve_form(op, 0, 0, PSI_PREC_FP64, S, 8, &form);
  if (s != PSI_OK) return s;
  if (form == kSegBands || form == kSegBins) S = 1;
  s = prepare_for(op, PSI_PREC_FP64, op->sched_items ? op->sched_items : kDefaultTileItems, S,
                  form, st);
  if (s != PSI_OK) return s;
  hipLaunchKernelGGL(k_make_z, dim3(grid_for(op->n)), dim3(kBlock), 0, st, s_vec, op->invden,
                     op->n, op->z_a);
  PassArgs a = base_args(op);
  a.x = op->z_a;
  a.s_new = psi_out;
  return run_pass(op, S, kFinal64, a, st);
}

// Times `reps` launches of a pass kind (see psi_pass_time); band layouts
// with column blocks of 2^wlog users and row blocks of `rows` rows (0: tuned
// or default).  A partial pass in the band layout is its band launches
// without the closing kernel, reported per launch.
psi_status pass_time_ex(psi_operator* op, int kind, int reps, int tile_items, int col_segments,
                        int seg_form, int wlog, int rows, double* mean_ms, hipStream_t st) {
  PSI_REQUIRE(mean_ms, "mean_ms must not be NULL");
  PSI_REQUIRE(reps >= 1, "reps must be >= 1");
  PSI_REQUIRE(kind >= PSI_PASS_STEP64 && kind <= PSI_PASS_PART32, "unknown pass kind");
  const bool part_only = kind == PSI_PASS_PART64 || kind == PSI_PASS_PART32;
  if (kind == PSI_PASS_PART64) kind = PSI_PASS_STEP64;
  if (kind == PSI_PASS_PART32) kind = PSI_PASS_STEP32;
  PSI_REQUIRE(kind != PSI_PASS_STEP64_W || op->val64,
              "the weighted pass needs an operator built with PSI_WEIGHTED_FP64");
  const int tile = tile_items ? tile_items : (op->sched_items ? op->sched_items : kDefaultTileItems);
  PSI_REQUIRE(tile_items_supported(tile), "unsupported tile_items");
  int S = 1;
  psi_status s = resolve_segments(op, col_segments, kind == PSI_PASS_STEP32 ? 4 : 8, &S);
  if (s != PSI_OK) return s;
  if (kind == PSI_PASS_STEP64_W) S = 1;
  const int prec = kind == PSI_PASS_STEP32 ? PSI_PREC_MIXED
                 : kind == PSI_PASS_STEP64_W ? PSI_PREC_FP64_WEIGHTED : PSI_PREC_FP64;
  int form = 0;
  s = resolve_form(op, seg_form, col_segments, prec, S, kind == PSI_PASS_STEP32 ? 4 : 8, &form);
  if (s != PSI_OK) return s;
  if (form == kSegBands || form == kSegBins) S = 1;
  PSI_REQUIRE(!part_only || (S > 1 && form != kSegBins) || form == kSegBands,
              "a partial pass needs col_segments > 1 or the band layout");
  if (form == kSegBands && !wlog && !rows) band_params(op, prec, &wlog, &rows);
  s = prepare(op, tile, S, form, st, wlog, rows);
  if (s != PSI_OK) return s;
  const int64_t n = op->n;
  hipLaunchKernelGGL(k_init64, dim3(grid_for(n)), dim3(kBlock), 0, st, nullptr, op->c, op->invden,
                     n, op->s_a, op->z_a);
  hipLaunchKernelGGL(k_init32, dim3(grid_for(n)), dim3(kBlock), 0, st, nullptr, op->c,
                     op->invden32, n, op->e_a, op->ze_a);
  PassArgs base = base_args(op);
  base.count_iter = 0;
  base.respect_done = 0;
  base.ctrl = op->ctrl + 1;
  base.r32 = op->c32;
  PassMode mode = kind == PSI_PASS_STEP64 ? kStep64
                : kind == PSI_PASS_STEP64_W ? kStep64W
                : kind == PSI_PASS_FINAL64 ? kFinal64 : kStep32;
  auto make = [&](int i) {
    PassArgs a = base;
    const bool even = (i & 1) == 0;
    if (mode == kStep32) {
      a.x = even ? op->ze_a : op->ze_b;
      a.e_old = even ? op->e_a : op->e_b;
      a.e_new = even ? op->e_b : op->e_a;
      a.ze_new = even ? op->ze_b : op->ze_a;
    } else if (mode == kFinal64) {
      a.x = op->z_a;
      a.s_new = op->s_b;
    } else {
      a.x = mode == kStep64W ? static_cast<const void*>(even ? op->s_a : op->s_b)
                             : static_cast<const void*>(even ? op->z_a : op->z_b);
      a.s_old = even ? op->s_a : op->s_b;
      a.s_new = even ? op->s_b : op->s_a;
      a.z_new = even ? op->z_b : op->z_a;
    }
    return a;
  };
  auto launch = [&](const PassArgs& a) {
    if (!part_only) return run_pass(op, S, mode, a, st);
    return form == kSegBands ? launch_pass_bands(op, mode, a, true, st)
                             : launch_part_seg(op, mode, a, st);
  };
  s = launch(make(0));
  if (s != PSI_OK) return s;
  EventPair tm;
  PSI_HIP_CHECK(hipEventCreate(&tm.a));
  PSI_HIP_CHECK(hipEventCreate(&tm.b));
  PSI_HIP_CHECK(hipEventRecord(tm.a, st));
  for (int i = 1; i <= reps; ++i) {
    s = launch(make(i));
    if (s != PSI_OK) return s;
  }
  PSI_HIP_CHECK(hipEventRecord(tm.b, st));
  PSI_HIP_CHECK(hipEventSynchronize(tm.b));
  float ms = 0.f;
  PSI_HIP_CHECK(hipEventElapsedTime(&ms, tm.a, tm.b));
  *mean_ms = static_cast<double>(ms) / reps;
  if (part_only && form == kSegBands) *mean_ms /= std::max(1, op->band_count);
  return PSI_OK;
}

psi_status pass_time(psi_operator* op, int kind, int reps, int tile_items, int col_segments,
                     int seg_form, double* mean_ms, hipStream_t st) {
  return pass_time_ex(op, kind, reps, tile_items, col_segments, seg_form, 0, 0, mean_ms, st);
}

// Times the loop kernels of a solve in `precision` for every supported tile
// size and column-segment count and keeps the fastest in the operator.
psi_status autotune(psi_operator* op, int precision, int reps, int* tile_items, int* col_segments,
                    int* seg_form, double* best_ms, hipStream_t st) {
  PSI_REQUIRE(precision >= PSI_PREC_FP64 && precision <= PSI_PREC_FP32, "unknown precision");
  PSI_REQUIRE(reps >= 0, "reps must be >= 0");
  PSI_REQUIRE(op->n_graphs == 1, "psi_autotune needs a single-graph operator");
  PSI_REQUIRE(precision != PSI_PREC_FP64_WEIGHTED || op->val64,
              "PSI_PREC_FP64_WEIGHTED needs an operator built with PSI_WEIGHTED_FP64");
  const int kind = precision == PSI_PREC_FP64 ? PSI_PASS_STEP64
                 : precision == PSI_PREC_FP64_WEIGHTED ? PSI_PASS_STEP64_W : PSI_PASS_STEP32;
  static const int kTiles[] = {1024, 1536, 2048, 3072, 4096};
  static const int kSegs[] = {1, 2, 4, 8};
  const int n_segs = precision == PSI_PREC_FP64_WEIGHTED ? 1 : 4;
  double best = 0.0;
  int best_tile = 0, best_S = 0, best_form = 0, best_wlog = 0, best_rows = 0;
  unsigned long long best_pace = 0;
  int tile_s1 = 0;  // fastest tile of the unsegmented pass (S = 1 is timed first)
  double best_s1 = 0.0;
  auto time_one = [&](int tile, int S, int form, int wlog, int rows, double* ms) -> psi_status {
    int r = reps;
    if (r == 0) {  // about 20 ms of passes per candidate, at least 3
      double one = 0.0;
      psi_status s = pass_time_ex(op, kind, 1, tile, S, form, wlog, rows, &one, st);
      if (s != PSI_OK) return s;
      r = static_cast<int>(std::min(50.0, std::max(3.0, 20.0 / std::max(one, 1e-3))));
    }
    return pass_time_ex(op, kind, r, tile, S, form, wlog, rows, ms, st);
  };
  // the fastest band layout on its own: the asynchronous sweeps run in it
  // whichever form wins the passes
  double band_best = 0.0;
  int band_wlog = 0, band_rows = 0;
  unsigned long long band_pace = 0;
  auto keep = [&](int tile, int S, int form, int wlog, int rows, double ms,
                  unsigned long long pace = 0) {
    if (form == kSegBands && (band_wlog == 0 || ms < band_best)) {
      band_best = ms;
      band_wlog = wlog;
      band_rows = rows;
      band_pace = pace;
    }
    if (best_tile == 0 || ms < best) {
      best = ms;
      best_tile = tile;
      best_S = S;
      best_form = form;
      best_wlog = wlog;
      best_rows = rows;
      best_pace = pace;
    }
  };
  for (int si = 0; si < n_segs; ++si) {
    const int S = kSegs[si];
    for (int tile : kTiles) {  // S = 1, or the tiled form of S segments
      double ms = 0.0;
      psi_status s = time_one(tile, S, S > 1 ? kSegTiles : 0, 0, 0, &ms);
      if (s != PSI_OK) return s;
      if (S == 1 && (tile_s1 == 0 || ms < best_s1)) {
        best_s1 = ms;
        tile_s1 = tile;
      }
      keep(tile, S, S > 1 ? kSegTiles : 0, 0, 0, ms);
    }
    if (S > 1) {  // the sliced form has no tiles: one timing, with the S = 1 tile kept
      double ms = 0.0;
      psi_status s = time_one(tile_s1, S, kSegSlices, 0, 0, &ms);
      if (s != PSI_OK) return s;
      keep(tile_s1, S, kSegSlices, 0, 0, ms);
    }
  }
  if (precision != PSI_PREC_FP64_WEIGHTED) {  // the band layout: column width x row-block size
    static const int kRows[] = {1024, 1280, 1536, 2048};
    int bw[4] = {0, 0, 0, 0};
    double bms[4] = {0.0, 0.0, 0.0, 0.0};
    op->band_pace_ticks = 0;
    for (int wlog = kBandMinLog; wlog <= kBandMaxLog; ++wlog)
      for (int ri = 0; ri < 4; ++ri) {
        double ms = 0.0;
        psi_status s = time_one(tile_s1, 1, kSegBands, wlog, kRows[ri], &ms);
        if (s != PSI_OK) return s;
        keep(tile_s1, 1, kSegBands, wlog, kRows[ri], ms);
        if (bw[ri] == 0 || ms < bms[ri]) {
          bw[ri] = wlog;
          bms[ri] = ms;
        }
      }
    // pacing of each row-block size at its faster column width: column block
    // c of a launch starts no earlier than c·pace, with pace a fraction of the
    // unpaced time per column block; waves drift apart less and their
    // gathers stay in L2 (the best pace is sharp and differs per layout)
    int dev = 0, khz = 0;
    PSI_HIP_CHECK(hipGetDevice(&dev));
    PSI_HIP_CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    int pr = -1;       // row-block size of the best paced candidate
    double pf = 0.0, pms = 0.0, pstep = 0.0;
    for (int ri = 0; ri < 4 && khz > 0; ++ri) {
      op->band_pace_ticks = 0;
      psi_status s = prepare(op, tile_s1, 1, kSegBands, st, bw[ri], kRows[ri]);
      if (s != PSI_OK) return s;
      if (op->band_B <= 1) break;
      const double step_us =
          bms[ri] * 1e3 / (double(std::max(1, op->band_count)) * op->band_B);
      for (double f : {0.4, 0.45, 0.5, 0.55, 0.6, 0.7}) {
        op->band_pace_ticks = static_cast<unsigned long long>(f * step_us * khz / 1e3);
        double ms = 0.0;
        s = time_one(tile_s1, 1, kSegBands, bw[ri], kRows[ri], &ms);
        if (s != PSI_OK) return s;
        keep(tile_s1, 1, kSegBands, bw[ri], kRows[ri], ms, op->band_pace_ticks);
        if (pr < 0 || ms < pms) {
          pr = ri;
          pf = f;
          pms = ms;
          pstep = step_us;
        }
      }
    }
    if (pr >= 0) {  // the optimum is sharp: finer paces around the best one
      op->band_pace_ticks = 0;
      psi_status s = prepare(op, tile_s1, 1, kSegBands, st, bw[pr], kRows[pr]);
      if (s != PSI_OK) return s;
      for (double df : {-0.025, -0.0125, 0.0125, 0.025}) {
        op->band_pace_ticks = static_cast<unsigned long long>((pf + df) * pstep * khz / 1e3);
        double ms = 0.0;
        s = time_one(tile_s1, 1, kSegBands, bw[pr], kRows[pr], &ms);
        if (s != PSI_OK) return s;
        keep(tile_s1, 1, kSegBands, bw[pr], kRows[pr], ms, op->band_pace_ticks);
      }
    }
    op->band_pace_ticks = 0;
    // the binned layout, when its count tables fit the workspace
    if (op->bins_val) {
      double ms = 0.0;
      psi_status s = time_one(tile_s1, 1, kSegBins, 0, 0, &ms);
      if (s == PSI_OK) keep(tile_s1, 1, kSegBins, 0, 0, ms);
      else if (s != PSI_EINVAL && s != PSI_ENOSPACE) return s;
    }
  }
  psi_status s = prepare(op, best_tile, best_S, best_form, st, best_wlog, best_rows);
  if (s != PSI_OK) return s;
  op->tuned_tile[precision] = best_tile;
  op->tuned_S[precision] = best_S;
  op->tuned_form[precision] = best_form;
  op->tuned_band_wlog[precision] = band_wlog;
  op->tuned_band_rows[precision] = band_rows;
  op->tuned_band_pace[precision] = band_pace;
  op->band_pace_ticks = best_form == kSegBands ? best_pace : 0ull;
  if (tile_items) *tile_items = best_tile;
  if (col_segments) *col_segments = best_S;
  if (seg_form) *seg_form = best_form;
  if (best_ms) *best_ms = best;
  return PSI_OK;
}

namespace {

// flag[0] = 1 if some user's activity is not the homogeneous λ = 1 − α,
// μ = α of the PageRank mode (within a few units in the last place)
__global__ void k_pr_check(const double* lam, const double* mu, int64_t n, double alpha,
                           int* flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double tl = 1.0 - alpha;
  const bool ok = fabs(lam[i] - tl) <= 8.0 * DBL_EPSILON * tl && fabs(mu[i] - alpha) <= 8.0 * DBL_EPSILON * alpha;
  if (!ok) *flag = 1;
}

__global__ void k_fill_f64(double* x, int64_t n, double v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_zero_i32(int* x) { *x = 0; }

}  // namespace

// PageRank mode (Sec. III-D): with λ_i = 1 − α and μ_i = α for every user the
// ψ-score is the PageRank vector of damping α (eq. pagerank_power).  In the
// power-method form the iterates are the power method's own: s_t = K·π_t with
// K = αN/(1 − α) satisfies s_t = Aᵀs_{t−1} + c from s_0 = K/N (π_0 uniform),
// so a step of ‖π_t − π_{t−1}‖₁ is one of ‖s_t − s_{t−1}‖₁ / K: the absolute
// (and ‖B‖-scaled) tolerances scale by K, the relative one does not; the
// returned (Bᵀs_t + d)/N is π_{t+1}.
psi_status pagerank(psi_operator* op, double alpha, const psi_params* prm, int power_method,
                    double* start, double* pi_out, psi_info* info, hipStream_t st) {
  PSI_REQUIRE(prm, "prm must not be NULL");
  PSI_REQUIRE(std::isfinite(alpha) && alpha > 0.0 && alpha < 1.0, "alpha must lie in (0, 1)");
  PSI_REQUIRE(op->n_graphs == 1, "the PageRank mode is for single-graph operators");
  PSI_REQUIRE(!power_method || start, "the power-method form needs a start vector buffer");
  PSI_REQUIRE(!power_method || prm->precision == PSI_PREC_FP64 ||
                  prm->precision == PSI_PREC_FP64_WEIGHTED,
              "the power-method form iterates in FP64");
  const int64_t n = op->n;
  if (n > 0) {
    int* flag = reinterpret_cast<int*>(op->scal + 7);
    int bad = 0;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, flag);
    hipLaunchKernelGGL(k_pr_check, dim3(grid_for(n)), dim3(kBlock), 0, st, op->lam, op->mu, n,
                       alpha, flag);
    PSI_HIP_CHECK(hipGetLastError());
    PSI_HIP_CHECK(hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    if (bad) {
      set_error("the PageRank mode needs lambda = 1 - alpha and mu = alpha for every user");
      return PSI_EINVAL;
    }
  }
  if (!power_method) return solve(op, prm, nullptr, pi_out, nullptr, info, st);
  psi_params p = *prm;
  const double K = alpha * static_cast<double>(n) / (1.0 - alpha);
  if (p.tol_mode != PSI_TOL_REL_L1) p.tol *= K;
  p.flags |= PSI_NO_FALLBACK;  // the start is the power method's, kept as given
  if (n > 0)
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kBlock), 0, st, start, n,
                       K / static_cast<double>(n));
  PSI_HIP_CHECK(hipGetLastError());
  return solve(op, &p, start, pi_out, nullptr, info, st);
}

}  // namespace psi
