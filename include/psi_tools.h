/*
 * psi_tools.h — schedule tuning, measurement and test hooks of the MI355X
 * Power-ψ library (psi.h holds the method's entry points).
 *
 * These calls do not compute ψ: they time the operator passes of
 * eq. (power_psi) in different launch schedules, pick the fastest for later
 * solves, measure the random-gather ceiling a pass is held to, and let a test
 * force the library's bounded waits to give up.  Conventions (status codes,
 * psi_last_error, devices, streams) are those of psi.h.
 */
#ifndef PSI_TOOLS_H
#define PSI_TOOLS_H

#include "psi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- operator pass kinds (for timing and tuning) -------------------------- */
#define PSI_PASS_STEP64     0  /* FP64 factored step: s' = c + μ⊙Σ_{j∈F(i)} s_j/den_j */
#define PSI_PASS_STEP64_W   1  /* FP64 weighted step: s' = c + Σ_j a_ji s_j           */
#define PSI_PASS_FINAL64    2  /* ψ = (λ⊙Σ_{j∈F(i)} s_j/den_j + d)/N                 */
#define PSI_PASS_STEP32     3  /* FP32 correction step: e' = r + μ⊙Σ e_j/den_j        */
#define PSI_PASS_PART64     4  /* only the per-segment partial kernel of STEP64       */
#define PSI_PASS_PART32     5  /* only the per-segment partial kernel of STEP32       */

/* Time `reps` back-to-back launches of one operator pass (the kernels a solve
 * runs in its loop: with col_segments > 1 the partial pass and the combine),
 * between two hipEvents recorded on `stream`, after one untimed launch.  Writes the mean duration of one launch in milliseconds to
 * *mean_ms (host).  tile_items, col_segments and seg_form as in psi_params.
 * Overwrites the operator's solve state.  Blocks until done. */
psi_status psi_pass_time(psi_operator* op, int32_t pass_kind, int32_t reps, int32_t tile_items,
                         int32_t col_segments, int32_t seg_form, double* mean_ms,
                         void* stream);

/* Random-gather probe: the access pattern of an operator pass without its
 * arithmetic, for the ceiling the pass is held to.  Workgroup b of `grid`
 * (a multiple of 8) streams its share of idx (device int32 [n_idx]) and
 * sums x[s·(n_x/S) + idx[k]] with s = (b mod 8) mod S — the column segment
 * its XCD group gathers from in a segmented pass (workgroups go to the 8
 * XCDs round-robin) — writing one sum per workgroup to out (device FP64
 * [grid]).  Indices are clamped into the segment.  x: device FP64 [n_x].
 * Times `reps` launches with hipEvents on `stream` after one untimed
 * launch; *mean_ms (host) is the mean.  Blocks. */
psi_status psi_gather_probe(const double* x, int64_t n_x, int32_t col_segments,
                            const int32_t* idx, int64_t n_idx, double* out, int32_t grid,
                            int32_t reps, double* mean_ms, void* stream);

/* Schedule autotuner.  Times `reps` back-to-back launches of the pass that
 * dominates a solve in `precision` (the FP64 step, the FP64 weighted step, or
 * the FP32 correction step for PSI_PREC_MIXED / PSI_PREC_FP32; with the
 * combine kernel when col_segments > 1) for every supported tile_items
 * (1024, 1536, 2048, 3072, 4096) and col_segments (1, 2, 4, 8; 1 only for
 * the weighted form), and for col_segments > 1 in both partial-pass forms
 * (the sliced form once, it has no tiles); outside the weighted form also
 * the band layout (both column widths at every row-block size, then each
 * row-block size paced) and the binned layout (when its count tables fit its
 * workspace); with hipEvents on `stream`.  It keeps the fastest in the
 * operator: later psi_solve calls in that precision whose psi_params leave
 * tile_items / col_segments / seg_form at 0 use it.  The fastest band layout
 * and pacing are kept as well, for calls that ask for the band layout
 * (psi_solve_async) whichever form won.  reps = 0 picks about 20 ms
 * of passes per candidate (at least 3).  Writes the choice and its mean pass
 * time (ms) to the host pointers, each of which may be NULL.  Overwrites the
 * operator's solve state; blocks.  Single-graph operators only. */
psi_status psi_autotune(psi_operator* op, int32_t precision, int32_t reps, int32_t* tile_items,
                        int32_t* col_segments, int32_t* seg_form, double* best_ms,
                        void* stream);

/* Scenario-batch autotuner (the multi-vector product over K activity
 * scenarios of psi_solve_batched).  Times the pass that dominates a batched
 * solve in `precision` (the FP64 step for PSI_PREC_FP64, the FP32 correction
 * step for PSI_PREC_MIXED, each with its gap kernels) over all K scenarios,
 * i.e. ceil(K / batch_tile) tile passes, on the operator's own rates in every
 * scenario, and keeps the fastest schedule in the operator for later
 * psi_solve_batched calls in that precision whose psi_params leave
 * batch_tile / batch_items / hub_chunk at 0.  Searched by coordinates:
 * scenarios per tile (8, 16, 32, 64 and K, at most 64), then merge-path items
 * per wave tile (128, 256, 512, 1024), then edges per long-row chunk (512,
 * 1024, 2048, 4096).  workspace: device, at least psi_batched_workspace_size
 * bytes for `precision` (overwritten).  reps = 0 picks about 20 ms of passes
 * per candidate (at least 3).  Writes the choice and the time of one pass
 * over all K scenarios (ms) to the host pointers (each may be NULL).
 * Single-graph operators; blocks. */
psi_status psi_autotune_batched(psi_operator* op, int32_t precision, int32_t n_scenarios,
                                void* workspace, size_t workspace_bytes, int32_t reps,
                                int32_t* batch_tile, int32_t* batch_items, int32_t* hub_chunk,
                                double* best_ms, void* stream);

/* Graph-batch autotuner (a multi-graph operator of psi_solve_batched).
 * Times whole graph batches in `precision` (PSI_PREC_FP64 or
 * PSI_PREC_MIXED) to the absolute L1 tolerance `tol`, without the final ψ
 * pass, for tile_items 1024, 2048, 3072, 4096 at col_segments 1, 2, 4, 8 (at
 * most 4 for PSI_PREC_MIXED) in the tiled form and, for col_segments > 1, the
 * sliced form; keeps the fastest in the operator for later graph batches in
 * that precision whose psi_params leave tile_items / col_segments / seg_form
 * at 0.  Whole solves are timed because graphs freeze as they converge and
 * only the tiled forms skip frozen graphs' gathers.  reps: timed solves per
 * candidate after one untimed (0 = 1).  *best_ms: the fastest solve's
 * device time.  Overwrites the operator's solve state; blocks. */
psi_status psi_autotune_graphs(psi_operator* op, int32_t precision, double tol, int32_t reps,
                               int32_t* tile_items, int32_t* col_segments, int32_t* seg_form,
                               double* best_ms, void* stream);

/* The band layout built on the operator (by a call that used PSI_SEG_BANDS or
 * by psi_autotune), for reports: column blocks of 2^col_log users (*col_blocks
 * of them), *row_blocks row blocks of at most *rows rows, run as *bands
 * launches per pass, *split_rows rows cut into pieces.  All zero when no band
 * layout is built.  Any out pointer may be NULL. */
psi_status psi_operator_band_info(const psi_operator* op, int32_t* col_log, int32_t* rows,
                                  int32_t* col_blocks, int32_t* row_blocks, int32_t* bands,
                                  int32_t* split_rows);

/* The binned layout built on the operator (by a call that used PSI_SEG_BINS
 * or by psi_autotune), for reports: *col_blocks follower blocks of
 * *block_users users, *bins bins (row blocks) of at most *rows rows,
 * *split_rows rows cut into pieces, *runs non-empty (follower block, bin)
 * pairs.  All zero when no binned layout is built.  Any out pointer may be
 * NULL. */
psi_status psi_operator_bins_info(const psi_operator* op, int32_t* block_users, int32_t* rows,
                                  int32_t* col_blocks, int32_t* bins, int32_t* split_rows,
                                  int64_t* runs);

/* Test hook for the recovery of a bounded wait that gives up.  The passes
 * hand partial sums between workgroups through slots that the reader waits
 * for (bounded); a wait that gives up makes the blocking call that saw it
 * return PSI_EDEVICE after emptying every slot and ticket of the operator, so
 * that later calls are unaffected.  With on = 1 every such wait on this
 * operator gives up at once (the partial it waits for is left in its slot);
 * on = 0 restores normal waits.  Blocks until set.  For tests only: a solve
 * with on = 1 and any partial handed between workgroups fails. */
psi_status psi_debug_force_slot_timeout(psi_operator* op, int32_t on);

#ifdef __cplusplus
}
#endif

#endif /* PSI_TOOLS_H */
