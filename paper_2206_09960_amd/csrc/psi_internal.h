// Internal declarations of the Power-ψ HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "psi.h"
#include "psi_tools.h"

namespace psi {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
void clear_error();

#define PSI_HIP_CHECK(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      psi::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));           \
      return PSI_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

#define PSI_REQUIRE(cond, msg)        \
  do {                                \
    if (!(cond)) {                    \
      psi::set_error(msg);            \
      return PSI_EINVAL;              \
    }                                 \
  } while (0)

// A pair of hipEvents destroyed with their scope (also on early error returns).
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() = default;
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// ---------------------------------------------------------------- constants
constexpr int kBlock = 256;            // threads of every operator-pass workgroup
constexpr int kMinTileItems = 1024;    // smallest merge-path tile (sizes the schedule)
constexpr int kDefaultTileItems = 2048;
constexpr int kHistLen = 1 << 16;      // device gap history entries
constexpr int kMaxGrid = 4096;         // largest grid of a pass kernel (64 groups of 64)
constexpr int kNoPass = 0x7fffffff;    // pass_id of a pass outside a deferred solve loop
// Cross-tile slots hold this signalling-NaN pattern while empty.  Every value
// a tile publishes is the result of floating-point arithmetic, which never
// produces a signalling NaN, so the pattern cannot collide with data.
constexpr unsigned long long kEmptySlot = 0x7FF4DEADBEEF0001ull;

// Validation bits raised by the build kernels.
enum : unsigned {
  kErrIndex = 1u,      // edge endpoint outside [0, n)
  kErrActivity = 2u,   // λ not finite/positive or μ not finite/non-negative
  kErrCrossGraph = 4u, // an edge joins two graphs of a multi-graph operator
  kErrSlotTimeout = 8u,  // a cross-tile slot was not filled in time (never expected)
};

// Message-passing aggregation: rows with more than kMpHubEdges entries are
// cut into chunks of kMpChunkEdges.
constexpr int kMpHubEdges = 64;
constexpr int kMpChunkEdges = 512;
struct MpHubs {
  int* hub_rows = nullptr;     // [max_hubs] rows with more than kMpHubEdges entries
  uint32_t* chunk0 = nullptr;  // [max_hubs + 1] first chunk of each hub
  int* chunk_hub = nullptr;    // [max_chunks] hub of each chunk
  int64_t n_hubs = -1;         // -1 until built
  int64_t n_chunks = 0;
};

// Device-side control block of one operator (one solve at a time).
struct Ctrl {
  // done and done_pass share one aligned 64-bit word, published together by
  // a single atomic store (publish_done) and read together (pass_cancelled), so
  // no reader sees done = 1 beside a stale done_pass
  int done;               // 1 once the gap met tol, max_iter hit or NaN seen
  int done_pass;          // pass whose workgroup 0 set done (-1: a kernel's tail or a
                          // separate decision); passes up to it still run in full
  unsigned int ticket;    // tiles finished in the current pass
  int iter;               // steps performed in the current solve
  int status;             // psi_status decided on the device
  unsigned int pending;   // gap pairs a deferred pass left for the next kernel to decide
  double gap;             // last gap in tol_mode units
  double l1;              // last ‖Δ‖₁
  double snorm;           // last ‖s_new‖₁
  double tol;
  int tol_mode;
  int max_iter;
  double bnorm;
  unsigned int err_flags;           // build validation and wait time-outs
  int force_timeout;      // set by the host (psi_debug_force_slot_timeout): every bounded
                          // wait gives up at once, to test the recovery path
  unsigned long long bnorm_bits;    // max over rows (bit pattern of a non-negative double)
  unsigned long long kappa_bits;
  unsigned long long n_self_loops;
  unsigned long long n_unique;
  unsigned long long n_no_leaders;
  unsigned long long max_row;
};
static_assert(offsetof(Ctrl, done) == 0 && offsetof(Ctrl, done_pass) == 4,
              "done and done_pass form the first 64-bit word of Ctrl");

// Arguments of one merge-path operator pass.  The pass gathers x over the
// follower lists of CSR(Aᵀ) and applies a per-row epilogue.
struct PassArgs {
  const int* row_ptr;
  const int* col;
  const int* tile_row;  // first row of each tile, [n_tiles + 1]
  int n_rows;
  int n_nnz;
  int n_tiles;
  int tile_items;
  const void* x;        // gathered vector (FP64 or FP32)
  const double* val64;  // per-edge weights (weighted form) or null
  // epilogue inputs / outputs
  const double* c;
  const double* mu;
  const double* invden;
  const double* lam;
  const double* d;
  const double* s_old;
  double* s_new;
  double* z_new;
  const float* r32;
  const float* mu32;
  const float* invden32;
  const float* e_old;
  float* e_new;
  float* ze_new;
  double inv_n;
  // cross-tile state
  double* part_open;   // [n_tiles] a tile's partial of its open last row (slot)
  double* gap_part;    // [2*grid] (Σ|Δ|, Σ|new|) of each workgroup (slot)
  double* gap_prev;    // deferred form: the previous pass's pairs, decided by workgroup 0
  int defer_gap;       // 1: write the pairs and leave the decision to the next kernel
  int pass_id;         // index of the pass in its solve loop (kNoPass outside one)
  double* gap_grp;     // [2*ceil(grid/64)] the same per group of 64 workgroups (slot)
  unsigned* grp_ticket;  // [ceil(grid/64)] arrivals per group (reset by its last)
  Ctrl* ctrl;
  double* hist;
  double* gap_out;      // optional plain copy of the gap (psi_step)
  const int* graph_of;  // block-diagonal operators: graph of each user
  const double* inv_ng; //   1/N of each user's graph
  const int* gdone;     //   graphs that met their tolerance (frozen)
  const int* gskip;     //   graphs frozen for a whole pass (both iterate buffers hold
                        //   their result): step passes may skip their gathers; NULL
                        //   in every other pass
  double* row_delta;    //   |s_new − s_old| of each user
  int count_iter;       // 1: the pass is a Power-ψ step that advances ctrl->iter
  int respect_done;     // 1: exit at once when ctrl->done is set
  int gs_sweep;         // 1: band-layout Gauss–Seidel sweep (psi_solve_async)
};

enum PassMode : int {
  kStep64 = 0,      // s_new = c + μ·Σ z_j, z_new = invden·s_new, gap
  kStep64W = 1,     // s_new = c + Σ a_ji s_j (weighted), gap
  kFinal64 = 2,     // ψ = (λ·Σ z_j + d)/N
  kStep32 = 3,      // e_new = r + μ·Σ ze_j, ze_new = invden·e_new, gap (FP32 storage)
  kPart64 = 4,      // y_s = Σ_{j∈F(i), j in segment s} x_j, x FP64 (partial pass)
  kPart32 = 5,      // same with x FP32, y_s stored FP32
  kStep64G = 6,     // kStep64 on a block-diagonal operator: per-graph freezing, |Δ| per row
  kFinal64G = 7,    // kFinal64 with 1/N of each user's own graph
  kStep32G = 8,     // kStep32 on a block-diagonal operator: per-graph freezing, |Δ| per row
};

// One column segment of CSR(Aᵀ): the followers in [lo, hi) of every row.
struct SegInfo {
  const int* row_ptr;   // [n_rows + 1], offsets into col (0-based per segment)
  const int* col;       // global follower ids
  const int* tile_row;  // merge-path schedule of this segment [n_tiles + 1] (tiled form)
  double* part_open;    // cross-tile slots [n_tiles] (tiled form)
  void* y;              // partial result [n_rows]
  int n_nnz;
  int n_tiles;
};

// The two forms of a segment's partial pass: merge-path tiles over the
// segment's CSR, or one lane per row over its sliced layout.
enum SegForm : int {
  kSegTiles = PSI_SEG_TILES,
  kSegSlices = PSI_SEG_SLICES,
  kSegBands = PSI_SEG_BANDS,  // column-blocked layout (psi_band.hip), not a segmentation
  kSegBins = PSI_SEG_BINS,    // binned two-launch pass (psi_bins.hip), not a segmentation
};

// Column-blocked ("band") layout: row blocks of at most 1024 or 2048 rows, each
// summed by one wave in LDS, over column blocks of 2^17 or 2^18 users.
constexpr int kBandMinLog = 17;
constexpr int kBandMaxLog = 18;
constexpr int kBandMaxCols = 1024;     // column blocks (LDS of the layout build)
constexpr int kBandWaveCap = 4096;     // waves of one band launch the capacities allow
constexpr int kBandMinEdges = 2048;
// rows per row block of the band layout: a wave's sums in LDS (8 B a row)
inline bool band_rows_supported(int r) { return r == 1024 || r == 1280 || r == 1536 || r == 2048; }    // smallest edge budget of a row block
constexpr int kBandFixGrid = 64;       // workgroups of the kernel that ends a band pass

struct BandBlock {
  int row_lo;  // first row
  int nrows;   // rows (1 for a piece of a split row)
  int piece;   // piece slot of a split row, -1 for whole rows
  int e_lo;    // first edge of the block in CSR(Aᵀ) (the next block's is its end)
};

// Arguments of one band launch.
struct BandArgs {
  const uint32_t* ent;      // entries (row in block << wlog | column in block)
  const uint32_t* toff;     // [n_blocks·B + 1] first entry of each (row block, column block)
  const BandBlock* blocks;  // [n_blocks + 1]
  double* piece;            // sums of the pieces of split rows
  double* pairs;            // (Σ|Δ|, Σ|new|) of each workgroup of the pass's band launches
  int B;
  int wlog;
  int first_block;          // first row block of this launch
  int n_blocks;             // row blocks of the whole layout
  int pair_base;            // first pair of this launch's workgroups
  int first_launch;         // 1 for the first launch of a pass (it decides a deferred gap)
  unsigned long long pace;  // wall-clock ticks between column-block starts (0 = no pacing)
  // Gauss–Seidel sweeps: users below fresh_below were updated earlier in this
  // sweep and are gathered from x_new, the others from the pass's x
  const void* x_new;
  int fresh_below;
};

// Arguments of the kernel that ends a band pass: the split rows, and the
// band launches' gap pairs reduced into this kernel's own.
struct BandFixArgs {
  const int4* split;        // {row, first piece, end piece, last block}
  const double* piece;
  const double* pairs;
  int n_split;
  int n_pairs;
};

// Binned ("propagation-blocked") pass, psi_bins.hip.  Followers are cut into
// column blocks of kBinsCols users, whose z a workgroup holds in LDS; leaders
// into bins (row blocks of at most kBinsRows rows, planned as the band
// layout's).  An expand kernel streams each column block's entries, reads z
// from LDS and writes the values in the order a bin reads them; a bin kernel
// then streams each bin's values and adds them to its rows' sums in LDS.
constexpr int kBinsCols = 20480;       // 160 KB of FP64 z: a CU's whole LDS
constexpr uint32_t kBinsColMask = 0x7FFFu;  // column in block (15 bits) of an expand word
constexpr int kBinsMaxB = 16384;        // column blocks (LDS of the layout build)
constexpr int kBinsRows = 1280;         // rows per bin (a wave's sums: 10 KB of LDS)
constexpr int kBinsMinEdges = 4096;     // smallest edge budget of a bin
constexpr int kBinsExpandWaves = 16;    // waves of an expand workgroup (one column block)
constexpr int kBinsWaves = 4;           // waves (bins) of a bin workgroup
constexpr uint32_t kBinsFirst = 0x8000u;  // entry flag: first entry of a (column block, bin) run

// Arguments of the two launches of a binned pass.
struct BinsArgs {
  const uint16_t* col;      // expand order: column in block | kBinsFirst, per column block
  const uint16_t* row;      // bin order: row in bin | kBinsFirst, per bin
  void* val;                // values in bin order (FP64, or FP32 in FP32 passes)
  const uint32_t* rdelta;   // per run: bin-order position − expand-order position (mod 2^32)
  const uint32_t* cs;       // [B + 1] first expand-order entry of each column block
  const int* task;          // [B · kBinsExpandWaves] run before each expand wave's first entry
  const uint32_t* bstart;   // [nb + 1] first bin-order entry of each bin
  const int* order;         // [nb] bins in launch order (most edges first)
  const BandBlock* blocks;  // [nb + 1] the bins (row blocks)
  double* piece;            // sums of the pieces of split rows
  double* pairs;            // (Σ|Δ|, Σ|new|) of each bin workgroup
  int B;                    // column blocks
  int per_xcd;              // column blocks per XCD (expand grid = 8 · per_xcd)
  int nb;                   // bins
  uint32_t runs;            // runs (rdelta entries)
  uint32_t m;               // entries
};

struct SegArgs {
  SegInfo seg[8];
  int S;
};

// Sliced form of a column segment, the layout its partial pass walks.  Rows
// are taken in windows of kSliceWindow; inside a window the rows with at most
// kSliceShort followers in the segment are ordered by length (longest first,
// ties by row) and packed 64 to a slice, one row per lane, their follower ids
// interleaved so that step k of all 64 lanes is one contiguous 256-byte run.
// Longer rows are cut into chunks of kSliceChunk edges, each summed by a whole
// wave; a row of several chunks is finished by the last of its chunks, which
// adds the chunk partials in chunk order.
constexpr int kSliceWindow = 4096;
constexpr int kSliceShort = 32;
constexpr int kSliceChunk = 64 * kSliceShort;

struct SliceDesc {
  int64_t off;  // short slice: first entry in slice_col; chunk: first edge in seg_col
  int len;      // short slice: steps (its longest row); chunk: edges
  int tag;      // >= 0: short slice, lane data at slice_row/slice_len[tag + lane];
                // < 0: chunk -1 - tag of slice_chunk
};

struct SliceSeg {
  const SliceDesc* slices;  // this segment's slices
  int n_slices;
  void* y;                  // partial result [n_rows]
};

struct SliceArgs {
  SliceSeg seg[8];
  int S;
  int respect_done;
  const void* x;              // gathered vector (FP64 or FP32)
  const int* row;             // [lane slots] row of each lane, -1 if none
  const unsigned char* len;   // [lane slots] followers of that row
  const int* col;             // interleaved follower ids of the short slices
  const int* seg_col;         // CSR of all segments (chunks index it)
  const int4* chunk;          // {row, slot or -1, first slot of the row, chunks of the row}
  double* part;               // chunk partials (slots, empty = kEmptySlot)
  unsigned* ticket;           // arrivals per multi-chunk row, indexed by its first slot
  Ctrl* ctrl;
  // a deferred gap of the previous pass, decided by workgroup 0
  double* gap_prev;
  double* hist;
  int count_iter;
  int defer_gap;
  int pass_id;
};


// ---------------------------------------------------------------- device helpers
// (shared by the pass and accelerated-solve kernels)

// Relaxed agent-scope store: visible to every workgroup of the device
// without a cache flush.
__device__ inline void st_agent(double* p, double x) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     static_cast<unsigned long long>(__double_as_longlong(x)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Fixed-order sum over the workgroup of two values; result in thread 0.
__device__ inline void block_sum2(double& a, double& b, double* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[2 * w] = a;
    sh[2 * w + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = (sh[0] + sh[2]) + (sh[4] + sh[6]);
    b = (sh[1] + sh[3]) + (sh[5] + sh[7]);
  }
  __syncthreads();
}

// done = 1 and done_pass in one relaxed agent-scope store of their shared
// word: every workgroup sees both or neither.
__device__ inline void publish_done(Ctrl* c, int done_pass) {
  const unsigned long long w = 1ull | (static_cast<unsigned long long>(
                                           static_cast<unsigned>(done_pass)) << 32);
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(&c->done), w, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// A pass of a solve loop that may stop at once: the device decided
// termination on an earlier pass (done_pass < pass_id), or, for the later
// kernels of a pass (inclusive), on this pass's own first kernel.  done and
// done_pass are read as one word.
__device__ inline bool pass_cancelled(const Ctrl* c, int pass_id, bool inclusive) {
  const unsigned long long w = __hip_atomic_load(
      reinterpret_cast<const unsigned long long*>(&c->done), __ATOMIC_RELAXED,
      __HIP_MEMORY_SCOPE_AGENT);
  if (!(w & 0xffffffffull)) return false;
  const int dp = static_cast<int>(static_cast<unsigned>(w >> 32));
  return inclusive ? dp <= pass_id : dp < pass_id;
}

// The termination decision on the reduced gap (thread 0): the iteration
// count, the gap in tol_mode units, its history, and done/status.
__device__ inline void decide_gap(Ctrl* c, double G, double S, double* hist, double* gap_out,
                                  int count_iter, int done_pass) {
  if (gap_out) *gap_out = G;
  if (!count_iter) return;
  double gap = G;
  if (c->tol_mode == PSI_TOL_BNORM) gap = G * c->bnorm;
  else if (c->tol_mode == PSI_TOL_REL_L1) gap = S > 0.0 ? G / S : G;
  const int it = c->iter + 1;
  c->iter = it;
  c->gap = gap;
  c->l1 = G;
  c->snorm = S;
  if (hist && it - 1 < kHistLen) hist[it - 1] = gap;
  int st = -1;
  if (!isfinite(gap)) st = PSI_ENUMERIC;
  else if (gap <= c->tol) st = PSI_OK;
  else if (it >= c->max_iter) st = PSI_ENOTCONV;
  if (st >= 0) {
    c->status = st;
    publish_done(c, done_pass);
  }
}

// Deferred gap, a whole workgroup of kBlock threads: the c->pending pairs a previous kernel
// left in `pairs` (complete, since that kernel has ended), summed in
// workgroup order — thread t a contiguous run, then a fixed tree — and
// decided as pass `pass_id`; the slots are emptied again.  Pairs of a pass
// that ran after the decision (its workgroups could not see it) are only
// emptied.
__device__ inline void take_deferred(Ctrl* c, double* pairs, double* hist, int count_iter,
                                     int pass_id, double* red) {
  const int n = static_cast<int>(c->pending);  // uniform
  if (n == 0) return;
  const int already = c->done;                  // uniform
  const int tid = threadIdx.x;
  const int per = (n + kBlock - 1) / kBlock;
  const int q_end = min(n, (tid + 1) * per);
  double G = 0.0, S = 0.0;
  for (int q = tid * per; q < q_end; ++q) {
    unsigned long long* p = reinterpret_cast<unsigned long long*>(pairs + 2 * q);
    G += __longlong_as_double(static_cast<long long>(
        __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    S += __longlong_as_double(static_cast<long long>(
        __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
    __hip_atomic_store(p, kEmptySlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, kEmptySlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum2(G, S, red);
  if (tid == 0) {
    c->pending = 0;
    if (!already) decide_gap(c, G, S, hist, nullptr, count_iter, pass_id);
  }
  __syncthreads();
}

}  // namespace psi

struct psi_operator {
  int device = 0;
  int64_t n = 0, m_in = 0, m = 0;
  int n_graphs = 1;
  uint32_t flags = 0;
  psi_operator_stats stats{};
  // persistent device arrays
  int* row_ptr = nullptr;   // CSR(Aᵀ): rows = leaders, cols = followers
  int* col = nullptr;
  int* fm_row_ptr = nullptr;  // CSR(A): rows = followers, cols = leaders L(j)
  int* fm_col = nullptr;
  int* graph_of = nullptr;     // graph of each user (n_graphs > 1)
  double* inv_ng = nullptr;    // 1/N of each user's graph (n_graphs > 1)
  double* row_delta = nullptr; // per-user |Δ| of the last pass (n_graphs > 1)
  // per-graph state (n_graphs > 1): G entries of the graphs' own iteration,
  // then G of the FP32 correction solve of a mixed-precision batch
  int* gdone = nullptr;
  int* gskip = nullptr;
  int* giter = nullptr;
  int* gstatus = nullptr;
  double* ggap = nullptr;
  double* gtol = nullptr;      // [G] tolerance of each graph's correction solve
  double *lam = nullptr, *mu = nullptr, *c = nullptr, *d = nullptr, *invden = nullptr;
  float *mu32 = nullptr, *invden32 = nullptr, *c32 = nullptr;
  double* val64 = nullptr;
  // solve state
  double *s_a = nullptr, *s_b = nullptr, *z_a = nullptr, *z_b = nullptr;
  float *e_a = nullptr, *e_b = nullptr, *ze_a = nullptr, *ze_b = nullptr, *r32 = nullptr;
  double *part_open = nullptr, *gap_part = nullptr, *gap_grp = nullptr;
  unsigned* grp_ticket = nullptr;
  int* tile_row = nullptr;
  int64_t max_tiles = 0;
  int sched_items = 0;   // tile size the schedule in tile_row was built for
  int n_tiles = 0;
  psi::Ctrl* ctrl = nullptr;   // [2]: outer solve, inner (FP32 correction) solve
  psi::Ctrl* host_ctrl = nullptr;  // pinned host mirror
  double* hist = nullptr;
  double* scal = nullptr;  // small FP64 device scratch (8 values)
  int64_t* graph_off = nullptr;  // device copy of node_offsets [n_graphs + 1]
  std::vector<int64_t> node_offsets;
  // column-segmented form of CSR(Aᵀ) and its sliced layout (built on first
  // use for a given S)
  int seg_S = 0;            // segments currently built (0 = none)
  int seg_items = 0;        // tile size of their merge-path schedules (0 = none)
  bool seg_sliced = false;  // their sliced layout is built
  int seg_form = 0;         // form the segmented passes of the current call use
  psi::SegInfo seg[8]{};
  int seg_slice0[9]{};      // first slice of each segment in slice_desc
  int64_t seg_off[9]{};     // first edge of each segment in seg_col
  // hub schedule of the message-passing aggregation, one per orientation
  // (0: CSR(Aᵀ), 1: CSR(A)); built on first use
  psi::MpHubs mp_hubs[2]{};
  int64_t mp_max_hubs = 0, mp_max_chunks = 0;
  // ‖Aᵀc + c − c‖₁ = ‖Aᵀc‖₁, the residual of the cold start (computed on first need)
  double rc_l1 = -1.0;
  // schedule chosen by psi_autotune, per precision (0 = not tuned)
  int tuned_tile[4]{};
  int tuned_S[4]{};
  int tuned_form[4]{};
  // scenario batches (psi_autotune_batched), per precision: scenarios per
  // tile, items per wave tile, edges per hub chunk (0 = not tuned)
  int tuned_batch_tile[4]{};
  int tuned_batch_items[4]{};
  int tuned_batch_chunk[4]{};
  // graph batches (psi_autotune_batched on a multi-graph operator), per
  // precision: tile items, column segments, partial-pass form (S = 0: not tuned)
  int tuned_graph_tile[4]{};
  int tuned_graph_S[4]{};
  int tuned_graph_form[4]{};
  int* seg_col = nullptr;       // [m]
  int* seg_row_ptr = nullptr;   // [8 * (n + 1)]
  int* seg_tile_row = nullptr;  // [max_seg_tiles + 8]
  double* seg_part_open = nullptr;  // [max_seg_tiles]
  int64_t max_seg_tiles = 0;
  double* seg_y = nullptr;      // [8 * n]
  uint32_t* seg_scan_tmp = nullptr;
  // sliced layout of the segments, sized for S = 8 (capacities below)
  psi::SliceDesc* slice_desc = nullptr;
  int* slice_row = nullptr;
  unsigned char* slice_len = nullptr;
  int* slice_col = nullptr;
  int4* slice_chunk = nullptr;
  double* slice_part = nullptr;
  unsigned* slice_ticket = nullptr;
  uint32_t* slice_plan = nullptr;  // per-window counts and their scans [5 * (8 * windows + 1)]
  int64_t cap_slices = 0, cap_lanes = 0, cap_entries = 0, cap_chunks = 0;
  // column-blocked (band) layout, built on first use
  bool band_built = false;
  int band_wlog = 0, band_rows = 0;  // column-block width 2^wlog, rows per row block
  int band_B = 0;                    // column blocks
  int band_nb = 0;                   // row blocks
  int band_waves = 0;                // row blocks (waves) per band launch
  int band_count = 0;                // band launches per pass
  int band_n_split = 0;              // rows cut into pieces
  std::vector<int> band_row0;        // first row of each band, and N
  std::vector<int> band_split_end;   // split rows whose last piece lies in bands 0..k
  unsigned long long band_pace_ticks = 0;  // pacing of the band launches (0 = none)
  int tuned_band_wlog[4]{}, tuned_band_rows[4]{};
  unsigned long long tuned_band_pace[4]{};
  uint32_t* band_ent = nullptr;      // [m]
  uint32_t* band_toff = nullptr;     // [cap_band_toff]
  psi::BandBlock* band_blocks = nullptr;  // [cap_band_blocks]
  int4* band_split = nullptr;        // [cap_band_blocks] {row, first piece, end piece, last block}
  double* band_piece = nullptr;      // [cap_band_blocks]
  double* band_pairs = nullptr;      // [2 * (cap_band_blocks / 4 + cap_band_blocks / 256 + 64)]
  uint32_t* band_scan_tmp = nullptr;
  int64_t cap_band_blocks = 0, cap_band_toff = 0, cap_band_cols = 0;
  // binned layout (psi_bins.hip), built on first use
  bool bins_built = false;
  int bins_B = 0;                    // column blocks of kBinsCols users
  int bins_nb = 0;                   // bins
  int bins_n_split = 0;              // rows cut into pieces
  int64_t bins_runs = 0;             // non-empty (column block, bin) runs
  void* bins_val = nullptr;          // [m] FP64 + 1 MiB (build scratch before the first pass)
  uint16_t* bins_col = nullptr;      // [m]
  uint16_t* bins_row = nullptr;      // [m]
  uint32_t* bins_rdelta = nullptr;   // [cap_bins_runs]
  uint32_t* bins_cs = nullptr;       // [cap_bins_cols + 1]
  uint32_t* bins_crun = nullptr;     // [cap_bins_cols + 1]
  int* bins_task = nullptr;          // [cap_bins_cols * kBinsExpandWaves]
  uint32_t* bins_bstart = nullptr;   // [cap_bins_blocks + 1]
  int* bins_order = nullptr;         // [cap_bins_blocks]
  psi::BandBlock* bins_blocks = nullptr;  // [cap_bins_blocks + 1]
  int4* bins_split = nullptr;        // [cap_bins_blocks]
  double* bins_piece = nullptr;      // [cap_bins_blocks]
  double* bins_pairs = nullptr;      // [2 * (cap_bins_blocks / kBinsWaves + 1)]
  int64_t cap_bins_blocks = 0, cap_bins_runs = 0, cap_bins_cols = 0;
  size_t cap_bins_val = 0;           // bytes of bins_val
};

namespace psi {
// Workspace layout shared by the size query and the build.
struct Layout {
  size_t persistent = 0;
  size_t scratch = 0;
};
Layout compute_layout(int64_t n, int64_t m_raw, int n_graphs, uint32_t flags);
void carve_persistent(psi_operator* op, char* base, int64_t m_raw, int n_graphs);

psi_status build_operator(psi_operator* op, const int32_t* follower, const int32_t* leader,
                          const double* lambda, const double* mu, const int64_t* node_offsets,
                          char* scratch, size_t scratch_bytes, hipStream_t stream);

psi_status ensure_schedule(psi_operator* op, int tile_items, hipStream_t stream);
// Build (or keep) the S-segment form of CSR(Aᵀ), then the layout the chosen
// partial-pass form walks: merge-path schedules of tile_items, or slices.
psi_status ensure_segments(psi_operator* op, int S, hipStream_t stream);
psi_status ensure_seg_tiles(psi_operator* op, int tile_items, hipStream_t stream);
psi_status ensure_seg_slices(psi_operator* op, hipStream_t stream);
// The column-blocked layout for column blocks of 2^wlog users and row blocks
// of at most `rows` rows (psi_band.hip), and the waves of one band launch.
psi_status ensure_bands(psi_operator* op, int wlog, int rows, hipStream_t stream);
int band_waves(int rows);
// The binned layout (psi_bins.hip).
psi_status ensure_bins(psi_operator* op, hipStream_t stream);
// One pass in the binned form: expand, bins, then the kernel that adds the
// pieces of split rows and ends the gap.
psi_status launch_pass_bins(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t stream);
// Layout of a call (requested, tuned, or from the gathered vector's size:
// band layout, or the partial-pass form of S segments) and the schedules and
// layouts its passes need; requested_S is the caller's col_segments.
psi_status resolve_form(const psi_operator* op, int requested, int requested_S, int precision,
                        int S, int bytes, int* form);
// Start of an FP32 correction solve of mixed precision from the FP64 step
// X → Y: r = Y − X rounded to FP32, e_0 = r (e_a, ze_a = e_0/den), and the
// inner control block (ctrl + 1) from the outer one's residual.
psi_status mixed_inner_begin(psi_operator* op, const double* Y, const double* X, double eta,
                             int max_iter, hipStream_t stream);
// X ← X + e and zX = X/den after a correction solve.
psi_status mixed_update(psi_operator* op, double* X, const float* e, double* zX,
                        hipStream_t stream);
psi_status prepare(psi_operator* op, int tile, int S, int form, hipStream_t stream);
// The same with the band layout's parameters (0: those built, else defaults).
psi_status prepare(psi_operator* op, int tile, int S, int form, hipStream_t stream, int wlog,
                   int rows);
// Band layout parameters a call uses: tuned ones for `precision`, else defaults.
void band_params(const psi_operator* op, int precision, int* wlog, int* rows);
// One pass in the band form: the band launches, then the kernel that adds the
// pieces of split rows and ends the gap (band_only: the band launches only).
psi_status launch_pass_bands(psi_operator* op, PassMode mode, const PassArgs& a, bool band_only,
                             hipStream_t stream);
// A pass in the operator's current form: bands, S column segments, or fused.
psi_status run_pass(psi_operator* op, int S, PassMode mode, const PassArgs& a, hipStream_t stream);
bool tile_items_supported(int t);
psi_status launch_pass(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t stream);
psi_status launch_pass_seg(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t stream);
// Only the per-segment partial kernel of a segmented kStep64 / kStep32 pass.
psi_status launch_part_seg(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t stream);
// Decide a deferred gap: the pairs in `pairs` left by the last pass on ctrl.
psi_status launch_gap_decide(Ctrl* ctrl, double* pairs, double* hist, int count_iter,
                             hipStream_t stream);
PassArgs base_args(psi_operator* op);

// Reads the wait-timeout bit of both control blocks (blocks the host).  When a
// bounded wait gave up, every cross-workgroup slot, ticket and gap slot is
// emptied again (a partial that arrived after its reader gave up would
// otherwise be read by a later pass), the bit is cleared, and PSI_EDEVICE is
// returned; otherwise PSI_OK.
psi_status check_waits(psi_operator* op, hipStream_t st);

psi_status solve_async(psi_operator* op, const psi_params* prm, const double* s0,
                       double* psi_out, double* s_out, psi_info* info, hipStream_t stream);
psi_status solve(psi_operator* op, const psi_params* prm, const double* s0, double* psi_out,
                 double* s_out, psi_info* info, hipStream_t stream);
psi_status pagerank(psi_operator* op, double alpha, const psi_params* prm, int power_method,
                    double* start, double* pi_out, psi_info* info, hipStream_t stream);
psi_status autotune(psi_operator* op, int precision, int reps, int* tile_items, int* col_segments,
                    int* seg_form, double* best_ms, hipStream_t stream);
psi_status autotune_batched(psi_operator* op, int precision, int K, void* ws, size_t ws_bytes,
                            int reps, int* batch_tile, int* batch_items, int* hub_chunk,
                            double* best_ms, hipStream_t stream);
psi_status autotune_graphs(psi_operator* op, int precision, double tol, int reps,
                           int* tile_items, int* col_segments, int* seg_form, double* best_ms,
                           hipStream_t stream);
psi_status gather_probe(const double* x, int64_t n_x, int S, const int32_t* idx, int64_t n_idx,
                        double* out, int grid, int reps, double* mean_ms, hipStream_t st);
psi_status anderson_workspace_size(const psi_operator* op, int depth, size_t* bytes);
psi_status solve_anderson_noalloc(psi_operator* op, const psi_params* prm, int depth,
                                  const double* s0, double* psi_out, double* s_out,
                                  psi_info* info, hipStream_t stream);
psi_status solve_anderson(psi_operator* op, const psi_params* prm, int depth, const double* s0,
                          double* psi_out, double* s_out, psi_info* info, void* ws,
                          size_t ws_bytes, hipStream_t st);

// Exclusive prefix sum of n uint32 (in may equal out); tile_sums needs
// scan_tile_count(n) + 1 entries; *total receives the sum.
psi_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tile_sums,
                              uint32_t* total, hipStream_t st);
int64_t scan_tile_count(int64_t n);
// Merge-path schedule: first row of each of n_tiles tiles of `items` path items.
psi_status build_schedule(const int* row_ptr, int64_t n, int64_t m, int items, int64_t n_tiles,
                          int* tile_row, hipStream_t st);

psi_status batched_workspace_size(const psi_operator* op, int n_scenarios, int precision,
                                  size_t* bytes);
psi_status solve_graphs(psi_operator* op, const psi_params* prm, double* psi_out, psi_info* infos,
                        hipStream_t st);
psi_status solve_batched(psi_operator* op, const psi_params* prm, int n_scenarios,
                         const double* lambda, const double* mu, double* psi_out, psi_info* infos,
                         void* ws, size_t ws_bytes, hipStream_t st);
psi_status solve_origins(psi_operator* op, const psi_params* prm, int K, const int32_t* origins,
                         double* p_out, double* psi_out, psi_info* infos, void* ws,
                         size_t ws_bytes, hipStream_t st);

// learned warm start (psi_mpnn.hip)
int64_t mpnn_param_count();
size_t model_state_size();
psi_status model_create(const float* params, int64_t n_params, uint32_t flags, void* state,
                        size_t state_bytes, hipStream_t st, psi_model** out);
psi_status model_destroy(psi_model* md);
psi_status model_get(const psi_model* md, int what, float* out, uint32_t flags, hipStream_t st);
psi_status mpnn_workspace_size(const psi_operator* op, int training, size_t* bytes);
psi_status mpnn_forward(psi_model* md, psi_operator* op, float* t_hat, double* s0, void* ws,
                        size_t ws_bytes, hipStream_t st);
psi_status mpnn_loss_backward(psi_model* md, psi_operator* op, const double* s_target,
                              double* loss, float* t_hat, void* ws, size_t ws_bytes,
                              hipStream_t st);
psi_status mpnn_adam_step(psi_model* md, double lr, double beta1, double beta2, double eps,
                          hipStream_t st);
}  // namespace psi
