/*
 * psi.h — C ABI of the MI355X (gfx950) Power-ψ library.
 *
 * The library computes the ψ-score of Arhachoui, Bautista, Danisch and
 * Giovanidis ("A Fast Algorithm for Ranking Users by their Influence in Online
 * Social Platforms", ASONAM 2022): given a directed follower graph and, per
 * user n, a posting rate λ_n and a re-posting rate μ_n (Sec. II), it solves the
 * single N-size system of eq. (ultimsol) by the power iteration of
 * Algorithm 2 (eq. power_psi) and returns ψ = (sᵀB + dᵀ)/N.
 *
 * Conventions shared by every entry point
 *   - Edge k is (follower[k], leader[k]): user follower[k] follows user
 *     leader[k] ((i, j) ∈ E means i follows j, Sec. II).  User ids are
 *     0 .. n_users-1.
 *   - Every function returns a psi_status; on failure psi_last_error() gives
 *     a message (thread-local, valid until the next call on that thread).
 *     No C++ exception crosses the ABI.
 *   - Device pointers are HIP device memory on the current device.  The
 *     library never allocates device memory: the caller passes workspaces
 *     whose sizes the *_workspace_size queries return.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     stream-ordered.  psi_build_operator and the solves block the calling
 *     host thread until their result is known, because when to stop depends
 *     on the data; psi_step and psi_final only enqueue.
 *   - One operator may not be used by two calls at the same time: the solve
 *     state lives in the operator's workspace.
 *   - Limits: n_users < 2^30, n_users + n_edges < 2^31 - 4096.
 */
#ifndef PSI_H
#define PSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum psi_status {
    PSI_OK = 0,
    PSI_EINVAL = 1,      /* bad argument or input (message says which)        */
    PSI_ENOTCONV = 2,    /* max_iter reached before the gap fell to tol       */
    PSI_ESTAGNATED = 3,  /* the gap stopped decreasing above tol              */
    PSI_ENUMERIC = 4,    /* NaN or Inf in the iteration                        */
    PSI_EDEVICE = 5,     /* a HIP runtime call failed or a bounded wait gave up */
    PSI_ENOSPACE = 6     /* a workspace is smaller than the size query said    */
} psi_status;

/* ---- operator build flags ------------------------------------------------ */
#define PSI_INPUT_HOST       0x1u  /* follower/leader/lambda/mu are host pointers   */
#define PSI_STRICT           0x2u  /* self-loops or repeated edges are an error     */
#define PSI_WEIGHTED_FP64    0x4u  /* also store a_ji per edge in FP64 (weighted form) */

/* ---- tolerance modes (how the gap of eq. eps_t is compared with tol) ------ */
#define PSI_TOL_ABS_L1  0  /* ‖s_t − s_{t−1}‖₁ ≤ tol   (eq. condition)            */
#define PSI_TOL_BNORM   1  /* ‖B‖·‖s_t − s_{t−1}‖₁ ≤ tol   (Algorithm 2 as printed) */
#define PSI_TOL_REL_L1  2  /* ‖s_t − s_{t−1}‖₁ / ‖s_t‖₁ ≤ tol                     */

/* ---- arithmetic of a solve ----------------------------------------------- */
#define PSI_PREC_FP64           0  /* FP64, factored operator (μ_i·Σ_j s_j/den_j)   */
#define PSI_PREC_FP64_WEIGHTED  1  /* FP64, per-edge a_ji (needs PSI_WEIGHTED_FP64) */
#define PSI_PREC_MIXED          2  /* FP32 correction solves + FP64 residual       */
#define PSI_PREC_FP32           3  /* FP32 iterate only (no refinement)            */

/* ---- solve flags ---------------------------------------------------------- */
#define PSI_NO_FALLBACK     0x1u  /* use s0 even if its residual is worse than c's */

/* ---- layout of the passes ---------------------------------------------------
 * Every layout computes the same sums (each row's followers added in a fixed
 * order, so results agree to rounding and each layout is bitwise repeatable).
 * Column-segmented passes (col_segments = S > 1) split the followers into S
 * segments, one per group of XCDs, and add the S partial sums per row; the
 * partial pass walks each segment in one of two layouts:
 *   TILES:  merge-path tiles of tile_items over the segment's CSR; suits a
 *           gathered vector whose segment share exceeds an XCD's L2;
 *   SLICES: one lane per row of at most 32 followers (rows ordered by length
 *           in windows of 4096, 64 to a slice), one wave per 2048-edge chunk
 *           of a longer row; suits a segment share that fits the L2.
 * BANDS is a layout of its own (col_segments is then ignored): followers are
 * cut into blocks of 2^17 or 2^18 users (1-2 MB of the FP64 iterate) and
 * leaders into row blocks of at most 1024 or 2048 rows, each summed by one
 * wave in LDS; the waves of one launch walk the follower blocks in step, so
 * their gathers hit L2 however large the graph; rows longer than a row block
 * are cut into pieces added in order afterwards.  It suits iterates larger
 * than the caches.
 * BINS is another layout of its own for iterates larger than the caches
 * (single-graph operators; FP64 factored, FP32 and final passes): followers
 * are cut into blocks of 20,480 users and leaders into bins of at most 1280
 * rows.  A pass is two streaming launches: the first reads each follower
 * block's slice of the iterate into LDS and writes one value per edge, in
 * the order the bins read them (8 bytes an edge, 4 in FP32 passes); the
 * second adds each bin's values to its rows' sums in LDS (propagation
 * blocking).  No gather leaves LDS, at the price of writing and reading the
 * per-edge values once per pass.  Its layout (12 bytes per edge and a run
 * table) is reserved in every single-graph operator's workspace.
 * 0 = the tuned form (psi_autotune), else SLICES when N·(8 or 4 bytes)/S is
 * at most 6 MB and TILES otherwise. */
#define PSI_SEG_TILES   1
#define PSI_SEG_SLICES  2
#define PSI_SEG_BANDS   3
#define PSI_SEG_BINS    4

typedef struct psi_operator psi_operator;

typedef struct psi_operator_stats {
    int64_t n_users;
    int64_t n_edges_in;      /* edges passed to the build                   */
    int64_t n_edges;         /* edges kept (M) after clean-up               */
    int64_t n_self_loops;    /* dropped self-loops                          */
    int64_t n_duplicates;    /* dropped repeated edges                      */
    int64_t n_no_leaders;    /* users with an empty newsfeed (zero rows)    */
    int64_t max_followers;   /* longest row of the pull operator            */
    int32_t n_graphs;
    int32_t flags;
    double b_norm;           /* ‖B‖ = max_j Σ_i b_ji (L1-induced, row vectors) */
    double kappa;            /* max_j Σ_i a_ji (< 1): contraction factor       */
} psi_operator_stats;

typedef struct psi_params {
    double tol;          /* ε > 0                                              */
    int32_t tol_mode;    /* PSI_TOL_*                                          */
    int32_t max_iter;    /* cap on Power-ψ iterations (A-products), > 0        */
    int32_t precision;   /* PSI_PREC_*                                         */
    int32_t check_every; /* host checks the gap every k steps; 0 = adaptive    */
    uint32_t flags;      /* PSI_NO_FALLBACK                                    */
    int32_t tile_items;  /* merge-path items per tile; 0 = library default     */
    int32_t col_segments;/* 1, 2, 4 or 8 column segments (one per XCD group);   */
                         /* 0 = chosen from N and the precision                */
    int32_t seg_form;    /* layout: PSI_SEG_TILES or PSI_SEG_SLICES (partial pass  */
                         /* of a segmented pass), PSI_SEG_BANDS, PSI_SEG_BINS;   */
                         /* 0 = tuned, else                                      */
                         /* from N and precision                                 */
    double inner_tol;    /* PSI_PREC_MIXED: each FP32 correction solve stops at
                            inner_tol·‖r‖₁ (0 = 2e-6) or at half the outer tol in L1
                            units, whichever is larger                           */
    int32_t band_col_log;/* PSI_SEG_BANDS: column blocks of 2^17 or 2^18 users;     */
                         /* 0 = tuned, else 18                                    */
    int32_t band_rows;   /* PSI_SEG_BANDS: rows per row block, 1024, 1280, 1536   */
                         /* or 2048;                                               */
                         /* 0 = tuned, else 2048                                  */
    int32_t batch_tile;  /* scenario batches: scenarios per tile, 1..64;          */
                         /* 0 = tuned, else 64                                    */
    int32_t batch_items; /* scenario batches: merge-path items per wave tile,     */
                         /* 128..8192; 0 = tuned, else 256                        */
    int32_t hub_chunk;   /* scenario batches: edges per chunk of a long row,      */
                         /* 512..8192; 0 = tuned, else 1024                       */
} psi_params;

typedef struct psi_info {
    int32_t status;           /* same value as the return code              */
    int32_t iterations;       /* Power-ψ steps t (FP64 A-products for MIXED) */
    int32_t spmv_passes;      /* all operator passes incl. the final Bᵀs one  */
    int32_t fp32_passes;      /* FP32 correction passes (MIXED / FP32)        */
    int32_t refinements;      /* FP64 residual evaluations (MIXED)            */
    int32_t used_s0;          /* 1 if the given s0 was used, 0 if c was       */
    int32_t col_segments;     /* column segments the passes used             */
    int32_t tile_items;       /* merge-path tile size the passes used        */
    double final_gap;         /* last gap in the tol_mode's units            */
    double final_l1_step;     /* last ‖s_t − s_{t−1}‖₁                        */
    double b_norm;
    double kappa;
    double err_bound_s;       /* κ/(1−κ)·‖s_t − s_{t−1}‖₁ ≥ ‖s − s_t‖₁        */
    double psi_gap_bound;     /* ‖s_t − s_{t−1}‖₁·‖B‖/N ≥ ‖ψ_t − ψ_{t−1}‖₁    */
    double device_ms;         /* time from first to last kernel of the solve  */
    int32_t seg_form;         /* PSI_SEG_* of the passes (0: fused, S = 1)    */
    int32_t batch_tile;       /* scenario batches: scenarios per tile         */
    int32_t hub_chunk;        /* scenario batches: edges per long-row chunk   */
} psi_info;

/* Library version string. */
const char* psi_version(void);

/* Message for the last failure on this thread ("" if none). */
const char* psi_last_error(void);

/* Sizes of the two device workspaces an operator build needs.
 *   persistent: holds the operator and its solve state for the operator's
 *               lifetime, including the layouts every pass form builds on
 *               first use (for a single-graph operator about 36 bytes per
 *               raw edge — CSR(Aᵀ), CSR(A), the segmented and sliced copies,
 *               the band entries, the binned layout's values, columns and
 *               rows — and about 220 bytes per user);
 *   scratch:    used only during psi_build_operator, free afterwards.
 * n_edges counts the raw edges, before self-loops and repeats are dropped. */
psi_status psi_operator_workspace_size(int64_t n_users, int64_t n_edges, int32_t n_graphs,
                                       uint32_t flags, size_t* persistent_bytes,
                                       size_t* scratch_bytes);

/* Build the Power-ψ operator (Sec. II, the definitions of A, b_i, C and d_i;
 * c and d are the diagonals of C and D, Sec. III-A) on the device:
 *   - drops self-loops and repeated edges (the graph is unweighted and has no
 *     self-loops, Sec. II), or fails with PSI_STRICT;
 *   - den_j = Σ_{ℓ∈L(j)} (λ_ℓ + μ_ℓ); a user with no leaders gets an empty
 *     (zero) row of A and B;
 *   - c_i = μ_i/(λ_i+μ_i), d_i = λ_i/(λ_i+μ_i);
 *   - the pull operator CSR(Aᵀ): row i lists the followers of i, ascending;
 *   - ‖B‖ and κ (largest row sums of B and A).
 * follower, leader: int32 [n_edges]; lambda, mu: FP64 [n_users]; host
 * pointers with PSI_INPUT_HOST, device pointers otherwise; not retained.
 * λ_i must be finite and > 0, μ_i finite and ≥ 0 (else PSI_EINVAL).
 * n_graphs > 1 stacks independent graphs block-diagonally: node_offsets
 * (host, int64 [n_graphs+1], 0 = first, n_users = last) gives each graph's
 * users and no edge may join two graphs.  n_graphs = 1 ignores node_offsets.
 * persistent/scratch: device buffers of at least the queried sizes.
 * *op receives a host handle (freed by psi_operator_destroy, which does not
 * free the workspaces).  Blocks until the build is done. */
psi_status psi_build_operator(int64_t n_users, int64_t n_edges, const int32_t* follower,
                              const int32_t* leader, const double* lambda, const double* mu,
                              int32_t n_graphs, const int64_t* node_offsets, uint32_t flags,
                              void* persistent, size_t persistent_bytes, void* scratch,
                              size_t scratch_bytes, void* stream, psi_operator** op);

psi_status psi_operator_destroy(psi_operator* op);

psi_status psi_operator_get_stats(const psi_operator* op, psi_operator_stats* out);

/* Device views of the built operator (read-only, valid while the persistent
 * workspace lives): row_ptr int32 [N+1] and col int32 [M] of CSR(Aᵀ); c, d,
 * inv_den (1/den_j, 0 for a user with no leaders) FP64 [N]. Any out pointer
 * may be NULL. */
psi_status psi_operator_views(const psi_operator* op, const int32_t** row_ptr,
                              const int32_t** col, const double** c, const double** d,
                              const double** inv_den);

/* Fill *p with the library defaults (tol 1e-8, PSI_TOL_ABS_L1, max_iter 10000,
 * PSI_PREC_FP64, adaptive checks). */
psi_status psi_params_default(psi_params* p);

/* Solve for ψ by Algorithm 2: s ← s0 (or c); repeat s ← Aᵀs + c until the gap
 * (tol_mode) is ≤ tol; then ψ = (Bᵀs + d)/N from the final s.
 *   s0:      device FP64 [N] start, or NULL for c.  Unless PSI_NO_FALLBACK,
 *            s0 is replaced by c when its residual ‖Aᵀs0 + c − s0‖₁ exceeds
 *            that of c (info->used_s0 says which was used);
 *   psi_out: device FP64 [N];
 *   s_out:   device FP64 [N] final s, or NULL;
 *   info:    host, may be NULL.
 * Returns PSI_ENOTCONV / PSI_ESTAGNATED / PSI_ENUMERIC with ψ of the last
 * iterate written. */
psi_status psi_solve(psi_operator* op, const psi_params* prm, const double* s0,
                     double* psi_out, double* s_out, psi_info* info, void* stream);

/* Asynchronous local updates (Sec. I names local-update methods such as Push
 * as the way beyond the power iteration): the same fixed point as psi_solve,
 * s = Aᵀs + c of eq. (power_psi), found by block Gauss–Seidel sweeps in a
 * fixed order.  The users are cut into consecutive bands (the band layout,
 * PSI_SEG_BANDS); in a sweep the bands are updated one after another, and
 * band k reads the users of bands 0..k−1 at their values from this sweep,
 * the others at the previous sweep's, so each user updates from fresher
 * values than Power-ψ's and fewer sweeps are needed.  The order is fixed, so
 * results are bitwise repeatable.  Stops when the sweep's change
 * ‖s_k − s_{k−1}‖₁ (tol_mode units) is at most tol (eq. condition); ψ =
 * (Bᵀs + d)/N from the final s (the last line of Algorithm 2).
 *   prm:    tol, tol_mode, max_iter (sweeps), check_every, band_col_log,
 *           band_rows as in psi_solve; precision must be PSI_PREC_FP64 and
 *           seg_form 0 or PSI_SEG_BANDS;
 *   s0:     device FP64 [N] start, or NULL for c (used as given);
 *   psi_out, s_out, info: as in psi_solve (info->iterations counts sweeps).
 * Single-graph operators; builds the band layout on first use; blocks. */
psi_status psi_solve_async(psi_operator* op, const psi_params* prm, const double* s0,
                           double* psi_out, double* s_out, psi_info* info, void* stream);

/* PageRank mode (Sec. III-D): with homogeneous activity λ_i = 1 − α and
 * μ_i = α the ψ-score is the PageRank vector with damping α
 * (eq. pagerank_power); users who follow nobody leak their mass.
 *   op:     a single-graph operator built with lambda = 1 − alpha and
 *           mu = alpha for every user (checked to a few ulps: PSI_EINVAL
 *           otherwise);
 *   alpha:  damping factor in (0, 1);
 *   prm:    as in psi_solve;
 *   power_method: 0 = plain Power-ψ from s_0 = c (psi_solve, tol on s);
 *           1 = the iterates of the PageRank power method itself:
 *           s_t = K·π_t with K = αN/(1 − α) solves s_t = Aᵀs_{t−1} + c from
 *           s_0 = K/N (π_0 uniform), so tol bounds ‖π_t − π_{t−1}‖₁ (the
 *           absolute and ‖B‖-scaled tolerances are applied to s as K·tol,
 *           the relative one as given) and the result (Bᵀs_t + d)/N is
 *           π_{t+1}; precision PSI_PREC_FP64 or PSI_PREC_FP64_WEIGHTED;
 *   start:  device FP64 [N], caller-owned scratch that receives s_0
 *           (power_method = 1 only; may be NULL otherwise);
 *   pi_out: device FP64 [N], the PageRank vector;
 *   info:   as in psi_solve.
 * Blocks until done, like psi_solve. */
psi_status psi_pagerank(psi_operator* op, double alpha, const psi_params* prm,
                        int32_t power_method, double* start, double* pi_out, psi_info* info,
                        void* stream);

/* One Power-ψ step (eq. power_psi), enqueued only:
 *   s_out = Aᵀ s_in + c,  *gap_out (device FP64 scalar, may be NULL)
 *   = ‖s_out − s_in‖₁.  precision PSI_PREC_FP64 or PSI_PREC_FP64_WEIGHTED.
 * s_in, s_out: device FP64 [N], distinct.  tile_items, col_segments and
 * seg_form as in psi_params (0 = default). */
psi_status psi_step(psi_operator* op, int32_t precision, const double* s_in, double* s_out,
                    double* gap_out, int32_t tile_items, int32_t col_segments,
                    int32_t seg_form, void* stream);

/* The last line of Algorithm 2, enqueued only: psi_out = (Bᵀ s + d)/N.
 * s, psi_out: device FP64 [N]. */
psi_status psi_final(psi_operator* op, const double* s, double* psi_out, void* stream);

/* Device workspace (bytes) of psi_solve_batched on this operator, for
 * precision PSI_PREC_FP64 or PSI_PREC_MIXED (scenario mode; the FP32
 * correction blocks add 28 bytes per user and scenario of a tile). */
psi_status psi_batched_workspace_size(const psi_operator* op, int32_t n_scenarios,
                                      int32_t precision, size_t* bytes);

/* Many independent Power-ψ solves in one call.
 * Scenario mode (n_scenarios = K ≥ 1, lambda and mu given): K activity
 * scenarios on the operator's graph — scenario k has rates
 * lambda[i*K + k], mu[i*K + k] (device FP64, user-major [N × K]) and its own
 * A, B, c, d (Sec. II) — solved together as one multi-vector pass per step
 * (scenarios in tiles of prm->batch_tile, 1..64: explicit, else as
 * psi_autotune_batched kept for the precision, else 64; prm->batch_items and
 * prm->hub_chunk likewise set the rows kernel's wave tiles and the long
 * rows' chunks; infos[k] reports the three).  Each scenario runs Algorithm 2 to its own
 * tolerance and is frozen afterwards; psi_out[i*K + k] (device FP64 [N × K])
 * is its ψ; infos[k] (host, may be NULL) its iteration count and gap.
 * The operator's own λ, μ are not used.
 * Graph mode (operator built with n_graphs = G > 1; n_scenarios = 1, lambda
 * and mu NULL): the G independent graphs of the block-diagonal operator are
 * solved together, one pass over all of them per step; each graph has its
 * own gap (over its users), stops at its own tolerance (and is frozen) and
 * its ψ uses its own N; psi_out (device [n_users]) holds every graph's ψ at
 * its users' positions, infos[g] (host, may be NULL) graph g's result;
 * prm->tile_items / col_segments / seg_form choose the pass as in
 * psi_solve (0: as psi_autotune_graphs kept for the precision, else two
 * segments with tiled partial passes from 10^6 users on, one fused pass
 * below).
 * Both modes also take PSI_PREC_MIXED: each refinement is one FP64
 * residual pass r = Aᵀs + c − s for every scenario (graph) — ‖r‖₁ is its
 * gap, the stopping test — then the FP32 correction solves e = Aᵀe + r of
 * all unfinished scenarios (graphs) together, each to
 * max(prm->inner_tol·‖r‖₁, tol / 2) (inner_tol 0 = 2e-6), and s ← s + e;
 * when a refinement stops shrinking some unfinished scenario's (graph's)
 * gap fourfold the batch finishes with FP64 steps.  infos[k].iterations counts the FP64 passes,
 * fp32_passes the correction passes.
 * Both modes: PSI_TOL_ABS_L1 only; returns the first non-OK scenario/graph
 * status, if any.
 * workspace: device, at least psi_batched_workspace_size bytes (0 in graph
 * mode: the operator's own workspace holds the state). */
psi_status psi_solve_batched(psi_operator* op, const psi_params* prm, int32_t n_scenarios,
                             const double* lambda, const double* mu, double* psi_out,
                             psi_info* infos, void* workspace, size_t workspace_bytes,
                             void* stream);

/* Anderson-accelerated Power-ψ.  The same fixed point as psi_solve, found
 * with fewer operator passes: each iteration is one Power-ψ pass
 * g = Aᵀx + c followed by Anderson mixing over the last `depth` residuals
 * (Anderson 1965; Walker & Ni 2011): γ = argmin ‖f_k − ΔF γ‖₂ with
 * f = g − x, x ← g − ΔG γ.  The stopping test is the pass's own gap
 * ‖g − x‖₁ ≤ tol in prm->tol_mode units, and s = g is returned, so the
 * result is a Power-ψ step of size at most tol (eq. condition), as in
 * Algorithm 2; ψ = (Bᵀs + d)/N.  depth in [1, 8].  PSI_PREC_FP64, or
 * PSI_PREC_MIXED: the refinement of psi_solve's PSI_PREC_MIXED (FP64
 * residual passes, the gap test and s = the last FP64 step as there), each
 * FP32 correction solve e = Aᵀe + r accelerated by the same mixing (FP32
 * window, FP64 dot products, an empty window per correction), to
 * max(prm->inner_tol·‖r‖₁, half the tolerance in L1 units); when a
 * refinement stops shrinking the gap fourfold, accelerated FP64 iterations
 * finish.  tile_items / col_segments as in psi_solve (the precision's
 * autotuned values used).  s0 (device FP64 [N], may be NULL = c) is the
 * start, used as given.  info->iterations counts FP64 passes (one per
 * iteration), fp32_passes the correction passes, info->refinements the
 * window restarts (FP64) or the correction solves (MIXED).  workspace:
 * device, at least
 * psi_anderson_workspace_size bytes (2·depth + 2 FP64 vectors of N plus
 * 130 KB).  Overwrites the operator's solve state; blocks. */
psi_status psi_anderson_workspace_size(const psi_operator* op, int32_t depth, size_t* bytes);
psi_status psi_solve_anderson(psi_operator* op, const psi_params* prm, int32_t depth,
                              const double* s0, double* psi_out, double* s_out, psi_info* info,
                              void* workspace, size_t workspace_bytes, void* stream);

/* psi_solve_anderson for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same solve, with its scratch (the ΔF/ΔG window, the
 * previous f and g, the partial sums and the mixing state) in a fixed device
 * array of 64 MiB inside the library instead of a caller workspace.  The
 * limit: (2·depth + 2)·8 bytes per user plus 130 KB must fit 64 MiB (about
 * 837,000 users at depth 4), else PSI_ENOSPACE with the sizes in the message.
 * The array is per device and shared by every call on that device: calls that
 * overlap on one GPU race (the solve blocks, so calls from one host thread do
 * not overlap).  It calls no hipMalloc or hipFree; every other argument and
 * result is as in psi_solve_anderson. */
psi_status psi_solve_anderson_noalloc(psi_operator* op, const psi_params* prm, int32_t depth,
                                      const double* s0, double* psi_out, double* s_out,
                                      psi_info* info, void* stream);

/* Per-origin newsfeed shares: Algorithm 1 (Power-NF, eq. fixpt_algo) for K
 * chosen origins at once.  For origin i, p_i solves p_i = A p_i + b_i
 * (eq. newsfeed: p_i^(j) is the share of user j's newsfeed that comes from
 * i), iterated from p_i = b_i until ‖p_i(t) − p_i(t−1)‖₁ ≤ tol (the
 * p-tolerance of Sec. V); each origin stops, and is frozen, on its own.
 * From it, q_i = C p_i + d_i (eq. wall: q_i^(j) = c_j p_i^(j), plus d_i at
 * j = i) is the share of j's wall from i, and ψ_i = (1/N) Σ_j q_i^(j)
 * (eq. psiscore).  This is the by-product Power-ψ skips: the influence of
 * one user on each other user.
 * origins: host int32 [K], user ids (repeats allowed).  p_out: device FP64
 * user-major [N × K] (p_out[j*K + k] = p_{origins[k]}^(j)), may be NULL.
 * psi_out: device FP64 [K], ψ of each origin.  infos: host [K], may be
 * NULL.  Only PSI_PREC_FP64 and PSI_TOL_ABS_L1; single-graph operators.
 * workspace: device, at least psi_batched_workspace_size bytes.  Blocks. */
psi_status psi_solve_origins(psi_operator* op, const psi_params* prm, int32_t n_origins,
                             const int32_t* origins, double* p_out, double* psi_out,
                             psi_info* infos, void* workspace, size_t workspace_bytes,
                             void* stream);

/* Schedule tuning, pass timing and the random-gather probe are declared in
 * psi_tools.h. */

/* ---- learned warm start ---------------------------------------------------
 * An extension of the method (the paper has none): a small message-passing
 * network predicts the fixed point s of eq. (power_psi) so that Algorithm 2
 * starts closer to it.  Since A ≥ 0, s ≥ c (Sec. II), and the network
 * predicts t̂ ≈ log(s/c) ≥ 0, giving s0 = c ⊙ exp(t̂).  Algorithm 2
 * converges from any start (the iteration contracts to the unique fixed
 * point), so a poor prediction costs iterations, never correctness, and
 * psi_solve keeps c when the residual of s0 is not smaller.
 *
 * The network, with F(i) the followers of i and den_j as in Sec. II:
 *   x0_i = [log λ_i, log(μ_i + 1e-12), c_i, d_i, log(1+|F(i)|),
 *           log(1+|L(i)|), log(1+den_i), 1]
 *   h = ReLU(x0 Win + bin)                                          (64)
 *   3 layers:  p_j = (h_j Wm)/den_j (32),  m_i = Σ_{j∈F(i)} p_j,
 *              h = ReLU([h | m] Wl + bl)                            (64)
 *   out = h·w_out + b_out,  t̂ = softplus(out)
 *   loss = mean over users with c_i > 0 of (t̂_i − log(s_i/c_i))²
 * Parameters: psi_mpnn_param_count() FP32 values, row-major, in the order
 * Win [8×64], bin [64], then per layer Wm [64×32], Wl [96×64], bl [64],
 * then w_out [64], b_out [1].  Wm, Wl and the activations h, p, m are used
 * in bfloat16 (round to nearest even), products accumulate in FP32.
 * Forward and backward are bitwise repeatable. */
typedef struct psi_model psi_model;

/* Number of FP32 parameters (25409). */
int64_t psi_mpnn_param_count(void);

/* Device bytes a model's state needs (parameters, Adam moments, gradient,
 * bf16 weight fragments). */
psi_status psi_model_state_size(size_t* bytes);

/* Creates a model on the current device.  params: n_params FP32 values in
 * the order above, host memory with PSI_INPUT_HOST in flags, else device
 * memory; copied.  state: caller-owned device memory of at least
 * psi_model_state_size bytes, kept by the model until psi_model_destroy
 * (Adam moments start at zero).  Blocks until the copy is done. */
psi_status psi_model_create(const float* params, int64_t n_params, uint32_t flags, void* state,
                            size_t state_bytes, void* stream, psi_model** model);
psi_status psi_model_destroy(psi_model* model);

/* Copies the current parameters / the last gradient (FP32 [param_count])
 * to out: host memory (blocks) with PSI_INPUT_HOST in flags, else device
 * memory (enqueued only). */
psi_status psi_model_params(const psi_model* model, float* out, uint32_t flags, void* stream);
psi_status psi_model_grad(const psi_model* model, float* out, uint32_t flags, void* stream);

/* Device workspace (bytes) of psi_mpnn_forward / psi_warmstart
 * (training = 0) and of psi_mpnn_loss_backward (training = 1) on this
 * operator: about 0.4 KB and 1.6 KB per user plus 2.2 bytes per edge. */
psi_status psi_mpnn_workspace_size(const psi_operator* op, int32_t training, size_t* bytes);

/* Forward pass on the operator's graph, enqueued only.  t_hat (device FP32
 * [N]) and s0 (device FP64 [N], = c ⊙ exp(t̂)) may each be NULL.
 * Model, operator and the current device must agree. */
psi_status psi_mpnn_forward(psi_model* model, psi_operator* op, float* t_hat, double* s0,
                            void* workspace, size_t workspace_bytes, void* stream);

/* The warm start s0_out = c ⊙ exp(t̂) (device FP64 [N]), enqueued only; pass
 * it to psi_solve as s0. */
psi_status psi_warmstart(psi_model* model, psi_operator* op, double* s0_out, void* workspace,
                         size_t workspace_bytes, void* stream);

/* Forward pass, loss against s_target (device FP64 [N], the fixed point
 * psi_solve returns in s_out) and backward pass; the gradient replaces the
 * model's stored one (read it with psi_model_grad).  *loss (host, may be
 * NULL; then the call only enqueues) receives the loss after the call
 * blocks.  t_hat (device FP32 [N], may be NULL) receives t̂. */
psi_status psi_mpnn_loss_backward(psi_model* model, psi_operator* op, const double* s_target,
                                  double* loss, float* t_hat, void* workspace,
                                  size_t workspace_bytes, void* stream);

/* One Adam step (Kingma & Ba, bias-corrected) on the stored gradient,
 * enqueued only.  Needs lr > 0, beta1, beta2 in [0, 1), eps > 0. */
psi_status psi_mpnn_adam_step(psi_model* model, double lr, double beta1, double beta2, double eps,
                              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PSI_H */
