// Batched Power-ψ: K activity scenarios (λ^k, μ^k) on one follower graph.
//
// Every scenario has its own A^k, B^k, c^k, d^k (Sec. II, the definitions of
// A, b_i, C, d_i), but all share the edge pattern, so one pass is a
// multi-vector product over CSR(Aᵀ): y_i^k = Σ_{j∈F(i)} s_j^k / den_j^k.  The
// iterates are stored user-major, [N × Kc] with Kc ≤ 64 scenarios per tile of
// the batch, so an edge gathers one contiguous Kc-vector and each lane of a
// wave owns one scenario.  Scenarios are independent solves of Algorithm 2:
// each has its own gap, stops at its own iteration (and is frozen afterwards)
// and gets ψ^k from its own final s^k.
//
// Mixed precision (scenario mode): the FP64 residual r^k = Aᵀs^k + c^k − s^k
// of every scenario comes from one FP64 pass (its L1 norm is the scenario's
// gap); the corrections e^k = Aᵀe^k + r^k are iterated together in FP32 on
// [N × Kc] FP32 blocks, each to its own tolerance η‖r^k‖₁, and s^k ← s^k + e^k.
// The fixed point is that of the FP64 iteration; when a refinement stops
// shrinking some scenario's residual fourfold, the batch finishes with plain
// FP64 steps.
//
// Origin mode: the newsfeed shares p_i of chosen origins i (Algorithm 1,
// Power-NF, eq. fixpt_algo) for K origins at once: one lane per origin, the
// same row tiles and hub chunks over CSR(A) (rows = followers j, columns =
// leaders ℓ), P ← A P + B from P = B, with (A P + B)_jk = (1/den_j)
// Σ_{ℓ∈L(j)} (μ_ℓ P_ℓk + λ_ℓ [ℓ = i_k]); each origin stops on its own
// p-tolerance ‖p_i(t) − p_i(t−1)‖₁ ≤ ε and ψ_i = (Σ_j c_j p_i^(j) + d_i) / N
// (eqs. wall and psiscore).
//
// Graph mode: G independent graphs stacked as one block-diagonal operator are
// solved together; each pass is an ordinary pass over the whole operator
// (fused, or column-segmented with a combine that applies the per-graph
// epilogue), then a per-graph kernel sums each graph's |Δ|, tests its own
// tolerance and freezes it.  A graph frozen for a whole pass holds its result
// in both iterate buffers, and the tiled passes skip the gathers of tiles
// that lie wholly in such graphs.
//
// Work split.  Rows (leaders) with at most kHubEdges followers are packed
// whole into wave tiles of about kWaveItems merge-path items; a wave sums its
// rows edge by edge in order.  Longer rows are cut into chunks of kChunkEdges
// edges; a workgroup reduces each chunk in a fixed order and a finishing
// kernel adds a row's chunks in chunk order.  A pass's per-scenario gap is
// summed in two fixed-order levels.  Every sum has a fixed order, so batched
// solves are bitwise repeatable.
#include <algorithm>
#include <cstdint>
#include <cmath>
#include <limits>
#include <vector>

#include "psi_internal.h"

namespace psi {

namespace {

constexpr int kWaveItems = 256;    // merge-path items per wave tile (default)
constexpr int kMinWaveItems = 128; // smallest wave tile the workspace holds
constexpr int kHubEdges = 256;     // rows longer than this are chunked
constexpr int kChunkEdges = 1024;  // edges per hub chunk (default)
constexpr int kMinChunkEdges = 512;   // smallest hub chunk the workspace holds
constexpr int kMaxChunkEdges = 8192;
constexpr int kMaxK = 64;          // scenarios per batch tile (at most one per lane)
constexpr int kHubFinGrid = 1024;  // largest grid of the hub-finishing kernel
constexpr int kGapParts = 64;      // first-level partials of a pass's gaps
constexpr int kGraphGapBlock = 1024;  // threads summing one graph's |Δ|

inline unsigned grid_for(int64_t n, int block = kBlock) {
  return static_cast<unsigned>((n + block - 1) / block);
}
inline size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

struct BatchCtrl {
  Ctrl c;          // global: done when every scenario is done
  int kdone[kMaxK];
  int kiter[kMaxK];
  int kstatus[kMaxK];
  double kgap[kMaxK];
  double ktol[kMaxK];  // each scenario's tolerance
};

// Workspace of one batch tile (reused for every tile of Kc scenarios).
struct BatchWs {
  double *lam, *mu, *c, *d, *invden;
  double *s_a, *s_b, *z_a, *z_b;
  int* row_tiles;      // [n_wtiles + 1]
  int* hub_rows;       // [max_hubs]
  int* hub_chunk0;     // [max_hubs + 1] first chunk of each hub
  int* chunk_row;      // [max_chunks]
  int* chunk_e0;       // [max_chunks]
  uint32_t* flags;     // [n + 1] scratch for the hub scan
  uint32_t* scan_tmp;
  double* chunk_part;  // [max_chunks × Kc]
  double* gap_blk;     // [kMaxGrid × Kc]
  double* gap_hub;     // [kHubFinGrid × Kc]
  double* gap_lvl;     // [kGapParts × Kc]
  BatchCtrl* ctrl;
  BatchCtrl* ctrl2;    // the FP32 correction solves (mixed precision)
  int* origin;         // [kMaxK] origins of the current tile (origin mode)
  // mixed precision only: μ, 1/den, r, e (×2), z_e = e/den (×2) as FP32 [N × Kc]
  float *mu32, *invden32, *r32, *e_a, *e_b, *ze_a, *ze_b;
  BatchCtrl* host_ctrl;  // not in the workspace
  int64_t n_wtiles, max_hubs, max_chunks;
};

size_t batch_layout(int64_t n, int64_t m, BatchWs* w, char* base, bool mixed) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(std::max<size_t>(bytes, 1));
    return p;
  };
  const int64_t n_wtiles = (n + m) / kMinWaveItems + 2;
  const int64_t max_hubs = m / (kHubEdges + 1) + 1;
  const int64_t max_chunks = m / kMinChunkEdges + max_hubs + 1;
  const size_t nk = 8 * size_t(n) * kMaxK;
  BatchWs t{};
  t.lam = (double*)take(nk);
  t.mu = (double*)take(nk);
  t.c = (double*)take(nk);
  t.d = (double*)take(nk);
  t.invden = (double*)take(nk);
  t.s_a = (double*)take(nk);
  t.s_b = (double*)take(nk);
  t.z_a = (double*)take(nk);
  t.z_b = (double*)take(nk);
  t.row_tiles = (int*)take(4 * size_t(n_wtiles + 1));
  t.hub_rows = (int*)take(4 * size_t(max_hubs));
  t.hub_chunk0 = (int*)take(4 * size_t(max_hubs + 1));
  t.chunk_row = (int*)take(4 * size_t(max_chunks));
  t.chunk_e0 = (int*)take(4 * size_t(max_chunks));
  t.flags = (uint32_t*)take(4 * size_t(n + 1));
  t.scan_tmp = (uint32_t*)take(4 * size_t(scan_tile_count(n + 1) + 8));
  t.chunk_part = (double*)take(8 * size_t(max_chunks) * kMaxK);
  t.gap_blk = (double*)take(8 * size_t(kMaxGrid) * kMaxK);
  t.gap_hub = (double*)take(8 * size_t(kHubFinGrid) * kMaxK);
  t.gap_lvl = (double*)take(8 * size_t(kGapParts) * kMaxK);
  t.ctrl = (BatchCtrl*)take(sizeof(BatchCtrl));
  t.ctrl2 = (BatchCtrl*)take(sizeof(BatchCtrl));
  t.origin = (int*)take(4 * size_t(kMaxK));
  if (mixed) {
    const size_t nk4 = 4 * size_t(n) * kMaxK;
    t.mu32 = (float*)take(nk4);
    t.invden32 = (float*)take(nk4);
    t.r32 = (float*)take(nk4);
    t.e_a = (float*)take(nk4);
    t.e_b = (float*)take(nk4);
    t.ze_a = (float*)take(nk4);
    t.ze_b = (float*)take(nk4);
  }
  t.n_wtiles = n_wtiles;
  t.max_hubs = max_hubs;
  t.max_chunks = max_chunks;
  if (w) *w = t;
  return off;
}

// ---------------------------------------------------------------- preparation
// λ^k, μ^k of this tile, user-major [N × Kc], from the caller's [N × K].
__global__ void k_bprep_act(const double* lam_in, const double* mu_in, int64_t n, int K, int k0,
                            int Kc, double* lam, double* mu, Ctrl* ctrl) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * Kc) return;
  const int64_t i = t / Kc;
  const int k = static_cast<int>(t % Kc);
  const double l = lam_in[i * K + k0 + k], m = mu_in[i * K + k0 + k];
  if (!(l > 0.0) || !isfinite(l) || !(m >= 0.0) || !isfinite(m))
    atomicOr(&ctrl->err_flags, kErrActivity);
  lam[t] = l;
  mu[t] = m;
}

// λ, μ of the operator's own users in every scenario of a tile (the timing
// runs of the batch autotuner: a pass's work does not depend on the rates).
__global__ void k_bprep_rep(const double* lam_op, const double* mu_op, int64_t n, int Kc,
                            double* lam, double* mu) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * Kc) return;
  lam[t] = lam_op[t / Kc];
  mu[t] = mu_op[t / Kc];
}

// den_j^k = Σ_{ℓ∈L(j)} (λ_ℓ^k + μ_ℓ^k) in ascending ℓ over CSR(A), one wave
// per follower j, lane k; then 1/den, c, d of user j.
__global__ void k_bprep_den(const int* fm_row_ptr, const int* fm_col, const double* lam,
                            const double* mu, int64_t n, int Kc, double* invden, double* c,
                            double* d) {
  const int64_t j = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int k = threadIdx.x & 63;
  if (j >= n || k >= Kc) return;
  double den = 0.0;
  for (int e = fm_row_ptr[j]; e < fm_row_ptr[j + 1]; ++e) {
    const int64_t l = fm_col[e];
    den += lam[l * Kc + k] + mu[l * Kc + k];
  }
  const int64_t t = j * Kc + k;
  invden[t] = den > 0.0 ? 1.0 / den : 0.0;
  const double lj = lam[t], mj = mu[t];
  c[t] = mj / (lj + mj);
  d[t] = lj / (lj + mj);
}

// FP32 copies of μ and 1/den for the correction solves.
__global__ void k_bprep32(const double* mu, const double* invden, int64_t total, float* mu32,
                          float* invden32) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  mu32[t] = static_cast<float>(mu[t]);
  invden32[t] = static_cast<float>(invden[t]);
}

// r = Y − X (the FP64 residual Aᵀs + c − s of X), rounded to FP32; e_0 = r.
__global__ void k_bprep_inner(const double* Y, const double* X, const float* invden32,
                              int64_t total, float* r32, float* e, float* ze) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const float r = static_cast<float>(Y[t] - X[t]);
  r32[t] = r;
  e[t] = r;
  ze[t] = invden32[t] * r;
}

// After a correction solve: X ← X + e for the scenarios still running; a
// finished scenario takes its final step Y (so X holds every finished
// scenario's result, which the next FP64 pass copies unchanged).
__global__ void k_bupdate(double* X, double* zX, const double* Y, const double* zY, const float* e,
                          const double* invden, const BatchCtrl* bc, int64_t total, int Kc) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  if (bc->kdone[t % Kc]) {
    X[t] = Y[t];
    zX[t] = zY[t];
  } else {
    const double v = X[t] + static_cast<double>(e[t]);
    X[t] = v;
    zX[t] = invden[t] * v;
  }
}

__global__ void k_binit(const double* c, const double* invden, int64_t total, double* s,
                        double* z) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  s[t] = c[t];
  z[t] = invden[t] * c[t];
}

// Wave tiles that hold whole rows: the merge-path row at diagonal b·items,
// moved past a row that straddles the diagonal.
__global__ void k_row_tiles(const int* row_ptr, int64_t n, int64_t m, int64_t items,
                            int64_t n_tiles, int* row_tiles) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b > n_tiles) return;
  const int64_t diag = std::min(b * items, n + m);
  int64_t lo = std::max<int64_t>(diag - m, 0), hi = std::min<int64_t>(diag, n);
  while (lo < hi) {
    const int64_t p = (lo + hi) >> 1;
    if (int64_t(row_ptr[p + 1]) <= diag - p - 1) lo = p + 1; else hi = p;
  }
  const int64_t e = diag - lo;
  int64_t r = lo;
  if (r < n && e > row_ptr[r]) ++r;
  row_tiles[b] = static_cast<int>(b == n_tiles ? n : r);
}

__global__ void k_hub_flags(const int* row_ptr, int64_t n, uint32_t* flags) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > n) return;
  flags[i] = (i < n && row_ptr[i + 1] - row_ptr[i] > kHubEdges) ? 1u : 0u;
}

__global__ void k_hub_list(const int* row_ptr, int64_t n, const uint32_t* pos, int chunk_edges,
                           int* hub_rows, uint32_t* nchunks) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int len = row_ptr[i + 1] - row_ptr[i];
  if (len > kHubEdges) {
    hub_rows[pos[i]] = static_cast<int>(i);
    nchunks[pos[i]] = static_cast<uint32_t>((len + chunk_edges - 1) / chunk_edges);
  }
}

__global__ void k_chunk_table(const int* row_ptr, const int* hub_rows, const uint32_t* chunk0,
                              int n_hubs, int chunk_edges, int* chunk_row, int* chunk_e0,
                              int* hub_chunk0) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= n_hubs) return;
  const int r = hub_rows[h];
  const int e0 = row_ptr[r], e1 = row_ptr[r + 1];
  int c = static_cast<int>(chunk0[h]);
  hub_chunk0[h] = c;
  for (int e = e0; e < e1; e += chunk_edges, ++c) {
    chunk_row[c] = r;
    chunk_e0[c] = e;
  }
}

// ---------------------------------------------------------------- passes
struct BArgs {
  const int* row_ptr;
  const int* col;
  int n_rows;
  int Kc;
  const int* row_tiles;
  int n_wtiles;
  const int* hub_rows;
  const int* hub_chunk0;
  int n_hubs;
  const int* chunk_row;
  const int* chunk_e0;
  int n_chunks;
  int chunk_edges;     // edges per hub chunk
  const double* z;     // gathered [N × Kc]
  const double* s_old;
  double* s_new;
  double* z_new;
  const double* c;
  const double* mu;
  const double* invden;
  const double* lam;
  const double* d;
  double inv_n;
  double* psi;         // final: psi[r * psi_ld + psi_col0 + k]
  int psi_ld;
  int psi_col0;
  double* chunk_part;
  double* gap_blk;
  double* gap_hub;
  double* gap_lvl;
  BatchCtrl* ctrl;
  const int* origin;   // origin mode: the origin of each lane
  // FP32 correction step: gathered z_e [N × Kc], r, μ, 1/den, e_old → e_new, z_e new
  const float* z32;
  const float* r32;
  const float* mu32;
  const float* invden32;
  const float* e_old;
  float* e_new;
  float* ze_new;
};

// Kernel modes: a scenario step, the scenarios' final ψ pass, an origin step,
// an FP32 correction step of the scenarios.
enum : int { kScen = 0, kScenFinal = 1, kOrig = 2, kScen32 = 3 };

// Epilogue inputs of row r for scenario k, loaded before the row's gathers.
// A scenario that has met its tolerance keeps its iterate, so it reads its s
// and z instead of the coefficients.
struct BRow {
  double a0, a1, a2, so;
};

template <int BM>
__device__ inline BRow bload(const BArgs& a, int r, int k, bool frozen) {
  const int64_t t = int64_t(r) * a.Kc + k;
  BRow in{0.0, 0.0, 0.0, 0.0};
  if constexpr (BM == kScenFinal) {
    in.a0 = a.lam[t];
    in.a1 = a.d[t];
  } else if constexpr (BM == kScen32) {
    in.so = a.e_old[t];
    if (frozen) {
      in.a0 = a.z32[t];
    } else {
      in.a0 = a.r32[t];
      in.a1 = a.mu32[t];
      in.a2 = a.invden32[t];
    }
  } else {
    in.so = a.s_old[t];
    if (frozen) {
      in.a0 = a.z[t];
    } else if constexpr (BM == kOrig) {  // shared 1/den, μ of the operator, indexed by user
      in.a1 = a.invden[r];
      in.a2 = a.mu[r];
    } else {
      in.a0 = a.c[t];
      in.a1 = a.mu[t];
      in.a2 = a.invden[t];
    }
  }
  return in;
}

// Row r's result for scenario k from its sum y.  Frozen scenarios store their
// kept iterate (and add no gap), so a wave's stores always cover whole lines.
template <int BM>
__device__ inline void bapply(const BArgs& a, int r, int k, const BRow& in, double y, bool frozen,
                              double& gap) {
  const int64_t t = int64_t(r) * a.Kc + k;
  if constexpr (BM == kScenFinal) {
    a.psi[int64_t(r) * a.psi_ld + a.psi_col0 + k] = (in.a0 * y + in.a1) * a.inv_n;
  } else if constexpr (BM == kScen32) {
    // e = r + μ y, z_e = e / den, in FP32
    float en = static_cast<float>(in.a0) + static_cast<float>(in.a1) * static_cast<float>(y);
    float zn = static_cast<float>(in.a2) * en;
    if (frozen) {
      en = static_cast<float>(in.so);
      zn = static_cast<float>(in.a0);
    }
    a.e_new[t] = en;
    a.ze_new[t] = zn;
    if (!frozen) gap += fabs(static_cast<double>(en) - in.so);
  } else {
    double sn, zn;
    if constexpr (BM == kOrig) {
      sn = in.a1 * y;   // p = y / den
      zn = in.a2 * sn;  // μ p, gathered by the next pass
    } else {
      sn = in.a0 + in.a1 * y;  // c + μ y
      zn = in.a2 * sn;         // s / den
    }
    if (frozen) {
      sn = in.so;
      zn = in.a0;
    }
    a.s_new[t] = sn;
    a.z_new[t] = zn;
    if (!frozen) gap += fabs(sn - in.so);
  }
}

// Origin mode adds λ_ℓ on the edge whose column is the lane's origin.
template <int BM>
__device__ inline double edge_term(const BArgs& a, int j, int k, int org, double lo) {
  if constexpr (BM == kScen32) {
    return static_cast<double>(a.z32[int64_t(j) * a.Kc + k]);
  } else {
    const double v = a.z[int64_t(j) * a.Kc + k];
    if constexpr (BM == kOrig) return j == org ? v + lo : v;
    return v;
  }
}

// Lanes of a wave in G groups of Kc (G·Kc ≤ 64): lane g·Kc + k works on
// scenario k of group g's row (or hub, or chunk); lanes past G·Kc shadow
// the last lane of the last group and store nothing.
template <int G>
struct LaneGroup {
  int g, k;
  bool active;
  __device__ LaneGroup(int lane, int Kc) {
    const int q = min(lane, G * Kc - 1);
    g = G == 1 ? 0 : q / Kc;
    k = q - g * Kc;
    active = lane < G * Kc;
  }
};

// Sum of the G groups' values of scenario `lane` (lane < Kc) over the four
// waves' rows of red, in wave then group order.
template <int G>
__device__ inline double sum_groups(double (*red)[64], int lane, int Kc) {
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w)
#pragma unroll
    for (int g = 0; g < G; ++g) t += red[w][g * Kc + lane];
  return t;
}

// Rows of at most kHubEdges followers: waves walk the wave tiles grid-stride.
// A wave reads the row ends of up to 63 rows in one load and, when those
// rows span at most kStage edges (no hub among them), stages their column
// indices in its slice of LDS; the G lane groups take consecutive rows; a
// row's epilogue inputs are loaded before its gathers, and up to 16 gathers
// per lane are in flight.  A row's edges are added one by one in order, so
// a row's sum does not depend on G.
template <int BM, int G>
__global__ __launch_bounds__(kBlock) void k_spmm_rows(BArgs a) {
  constexpr bool FINAL = BM == kScenFinal;
  constexpr int kB = 16;       // gathers in flight per lane
  constexpr int kStage = 256;  // staged column indices per wave
  __shared__ double red[kBlock / 64][64];
  __shared__ int s_col[kBlock / 64][kStage];
  if (!FINAL && a.ctrl->c.done) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const LaneGroup<G> lg(lane, a.Kc);
  const int k = lg.k;
  const bool frozen = !FINAL && a.ctrl->kdone[k];
  const int org = BM == kOrig ? a.origin[k] : -1;
  const double lo = BM == kOrig ? a.lam[org] : 0.0;
  int* cw = s_col[wave];
  double gap = 0.0;
  const int stride = gridDim.x * (kBlock / 64);
  for (int tile = blockIdx.x * (kBlock / 64) + wave; tile < a.n_wtiles; tile += stride) {
    const int r0 = a.row_tiles[tile], r1 = a.row_tiles[tile + 1];
    for (int rb = r0; rb < r1; rb += 63) {
      const int nb = min(63, r1 - rb);
      const int rp = a.row_ptr[rb + min(lane, nb)];  // row rb + i spans [rp_i, rp_{i+1})
      const int E0 = __builtin_amdgcn_readlane(rp, 0);
      const int E1 = __builtin_amdgcn_readlane(rp, nb);
      const bool staged = E1 - E0 <= kStage;
      if (staged && E1 > E0) {
        int t[kStage / 64];  // all four loads in flight, then the LDS writes
#pragma unroll
        for (int q = 0; q < kStage / 64; ++q) t[q] = a.col[min(E0 + q * 64 + lane, E1 - 1)];
#pragma unroll
        for (int q = 0; q < kStage / 64; ++q) cw[q * 64 + lane] = t[q];
      }
      // y of a row from its column indices idx(0 .. len), in order
      auto row_sum = [&](int len, auto idx) -> double {
        double y = 0.0;
        for (int u0 = 0; u0 < len; u0 += kB) {
          int jj[kB];
#pragma unroll
          for (int u = 0; u < kB; ++u) jj[u] = idx(min(u0 + u, len - 1));
          double v[kB];
#pragma unroll
          for (int u = 0; u < kB; ++u) {
            v[u] = 0.0;
            if (u0 + u < len) v[u] = edge_term<BM>(a, jj[u], k, org, lo);
          }
#pragma unroll
          for (int u = 0; u < kB; ++u) y += v[u];
        }
        return y;
      };
      if constexpr (G == 1) {
        if (staged) {
          // The block's edges as one stream, kB gathers in flight across row
          // boundaries; a row's sum still adds its edges one by one in order
          // (the same bits as row by row), and each row's epilogue inputs are
          // loaded while the row before it is summed.  A staged block holds
          // no hub (at most kStage <= kHubEdges edges in all).
          int i = 0;
          int bnd = __builtin_amdgcn_readlane(rp, 1);  // end of row i
          BRow cur = bload<BM>(a, rb, k, frozen);
          BRow nxt = nb > 1 ? bload<BM>(a, rb + 1, k, frozen) : BRow{0.0, 0.0, 0.0, 0.0};
          double acc = 0.0;
          auto flush = [&]() {
            if (lane < a.Kc) bapply<BM>(a, rb + i, k, cur, acc, frozen, gap);
            acc = 0.0;
            ++i;
            cur = nxt;
            if (i + 1 < nb) nxt = bload<BM>(a, rb + i + 1, k, frozen);
            bnd = __builtin_amdgcn_readlane(rp, min(i + 1, nb));
          };
          for (int q0 = E0; q0 < E1; q0 += kB) {
            int jj[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) jj[u] = cw[min(q0 + u, E1 - 1) - E0];
            double v[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
              v[u] = 0.0;
              if (q0 + u < E1) v[u] = edge_term<BM>(a, jj[u], k, org, lo);
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
              const int q = q0 + u;
              if (q >= E1) break;  // uniform
              while (q >= bnd) flush();
              acc += v[u];
            }
          }
          while (i < nb) flush();
          continue;
        }
      }
      for (int i0 = 0; i0 < nb; i0 += G) {
        int i, e0, len;
        if constexpr (G == 1) {  // one row per wave: its bounds are uniform
          i = i0;
          e0 = __builtin_amdgcn_readlane(rp, i0);
          len = __builtin_amdgcn_readlane(rp, i0 + 1) - e0;
          if (len > kHubEdges) continue;  // finished by the hub kernels
        } else {
          i = min(i0 + lg.g, nb);  // i == nb: past the block, an empty row
          e0 = __shfl(rp, i, 64);
          len = __shfl(rp, min(i + 1, nb), 64) - e0;
          if (len > kHubEdges) len = -1;  // finished by the hub kernels
        }
        const bool mine = i < nb && len >= 0;
        const int r = rb + min(i, nb - 1);
        const BRow in = mine ? bload<BM>(a, r, k, frozen) : BRow{0.0, 0.0, 0.0, 0.0};
        const int n_e = max(len, 0);
        const double y = staged ? row_sum(n_e, [&](int q) { return cw[e0 - E0 + q]; })
                                : row_sum(n_e, [&](int q) { return a.col[e0 + q]; });
        if (lg.active && mine) bapply<BM>(a, r, k, in, y, frozen, gap);
      }
    }
  }
  if constexpr (!FINAL) {
    red[wave][lane] = gap;
    __syncthreads();
    if (wave == 0 && lane < a.Kc)
      a.gap_blk[int64_t(blockIdx.x) * a.Kc + lane] = sum_groups<G>(red, lane, a.Kc);
  }
}

// G hub chunks per workgroup, one per lane group: wave w sums its group's
// chunk's edges e0+w, e0+w+4, ...; the four wave sums are added in wave
// order (the same order for every G).
template <int BM, int G>
__global__ __launch_bounds__(kBlock) void k_spmm_hub_chunk(BArgs a) {
  __shared__ double red[kBlock / 64][64];
  if (BM != kScenFinal && a.ctrl->c.done) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const LaneGroup<G> lg(lane, a.Kc);
  const int k = lg.k;
  const int org = BM == kOrig ? a.origin[k] : -1;
  const double lo = BM == kOrig ? a.lam[org] : 0.0;
  const int ch = static_cast<int>(blockIdx.x) * G + lg.g;
  const bool mine = ch < a.n_chunks;
  const int chc = min(ch, a.n_chunks - 1);
  const int r = a.chunk_row[chc];
  const int e0 = a.chunk_e0[chc];
  const int e1 = mine ? min(e0 + a.chunk_edges, a.row_ptr[r + 1]) : e0;
  double y = 0.0;
  int e = e0 + wave;
  for (; e + 28 < e1; e += 32) {
    int j[8];
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) j[u] = a.col[e + 4 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = edge_term<BM>(a, j[u], k, org, lo);
#pragma unroll
    for (int u = 0; u < 8; ++u) y += v[u];
  }
  for (; e < e1; e += 4) y += edge_term<BM>(a, a.col[e], k, org, lo);
  red[wave][lane] = y;
  __syncthreads();
  if (wave == 0 && lg.active && mine)
    a.chunk_part[int64_t(ch) * a.Kc + k] =
        ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Hub rows: lane group g of wave w of workgroup b finishes hubs
// (4b + w)·G + g, then every 4·G·grid further (a row's chunks in chunk
// order, 16 loads in flight, then the epilogue).  A lane adds the gaps of
// its hubs in order; the workgroup adds its waves and groups in order.
template <int BM, int G>
__global__ __launch_bounds__(kBlock) void k_spmm_hub_finish(BArgs a) {
  constexpr bool FINAL = BM == kScenFinal;
  __shared__ double red[kBlock / 64][64];
  if (!FINAL && a.ctrl->c.done) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const LaneGroup<G> lg(lane, a.Kc);
  const int k = lg.k;
  const bool frozen = !FINAL && a.ctrl->kdone[k];
  double gap = 0.0;
  const int stride = gridDim.x * (kBlock / 64) * G;
  for (int h = (blockIdx.x * (kBlock / 64) + wave) * G + lg.g; h < a.n_hubs; h += stride) {
    const int r = a.hub_rows[h];
    const BRow in = bload<BM>(a, r, k, frozen);
    const int c0 = a.hub_chunk0[h], c1 = a.hub_chunk0[h + 1];
    double y = 0.0;
    for (int ch = c0; ch < c1; ch += 16) {
      double p[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) p[u] = a.chunk_part[int64_t(min(ch + u, c1 - 1)) * a.Kc + k];
#pragma unroll
      for (int u = 0; u < 16; ++u) y += ch + u < c1 ? p[u] : 0.0;
    }
    if (lg.active) bapply<BM>(a, r, k, in, y, frozen, gap);
  }
  if constexpr (!FINAL) {
    red[wave][lane] = gap;
    __syncthreads();
    if (wave == 0 && lane < a.Kc)
      a.gap_hub[int64_t(blockIdx.x) * a.Kc + lane] = sum_groups<G>(red, lane, a.Kc);
  }
}

// Per-scenario gaps, first level: workgroup p sums a contiguous range of the
// rows kernel's and then the hub kernel's per-workgroup partials (wave w
// takes entries w, w + 4, ... of the range in order; then waves in order).
__global__ __launch_bounds__(kBlock) void k_batch_gap_part(BArgs a, int n_blk, int n_hblk) {
  __shared__ double red[kBlock / 64][kMaxK];
  if (a.ctrl->c.done) return;  // uniform
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t total = int64_t(n_blk) + n_hblk;
  const int b0 = static_cast<int>(total * blockIdx.x / gridDim.x);
  const int b1 = static_cast<int>(total * (blockIdx.x + 1) / gridDim.x);
  double g = 0.0;
  if (lane < a.Kc) {
#pragma unroll 4
    for (int b = b0 + wave; b < b1; b += 4)
      g += b < n_blk ? a.gap_blk[int64_t(b) * a.Kc + lane]
                     : a.gap_hub[int64_t(b - n_blk) * a.Kc + lane];
  }
  red[wave][lane] = g;
  __syncthreads();
  if (wave == 0 && lane < a.Kc)
    a.gap_lvl[int64_t(blockIdx.x) * a.Kc + lane] =
        ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Second level, one wave: lane k adds scenario k's kGapParts partials in
// order, tests the tolerance and freezes; done when every scenario is done.
__global__ __launch_bounds__(64) void k_batch_gap(BArgs a) {
  BatchCtrl* bc = a.ctrl;
  if (bc->c.done) return;  // uniform
  const int lane = threadIdx.x;
  int done = 1;
  if (lane < a.Kc) {
    double G = 0.0;
#pragma unroll 8
    for (int p = 0; p < kGapParts; ++p) G += a.gap_lvl[int64_t(p) * a.Kc + lane];
    if (!bc->kdone[lane]) {
      const int it = bc->kiter[lane] + 1;
      bc->kiter[lane] = it;
      bc->kgap[lane] = G;
      if (!isfinite(G)) {
        bc->kdone[lane] = 1;
        bc->kstatus[lane] = PSI_ENUMERIC;
      } else if (G <= bc->ktol[lane]) {
        bc->kdone[lane] = 1;
        bc->kstatus[lane] = PSI_OK;
      } else if (it >= bc->c.max_iter) {
        bc->kdone[lane] = 1;
        bc->kstatus[lane] = PSI_ENOTCONV;
      }
    }
    done = bc->kdone[lane];
  }
  const int all = __all(done);
  if (lane == 0) {
    bc->c.iter += 1;
    if (all) bc->c.done = 1;
  }
}

__global__ void k_bctrl_init(BatchCtrl* bc, double tol, int max_iter) {
  bc->c = Ctrl{};
  bc->c.tol = tol;
  bc->c.max_iter = max_iter;
  for (int k = 0; k < kMaxK; ++k) {
    bc->kdone[k] = 0;
    bc->kiter[k] = 0;
    bc->kstatus[k] = PSI_OK;
    bc->kgap[k] = 0.0;
    bc->ktol[k] = tol;
  }
}

// Control block of a correction solve: scenario k runs to η·‖r^k‖₁ (its last
// FP64 gap), or to half its own L1 tolerance when that is larger (solving the
// correction below what the outer test asks buys nothing); scenarios already
// finished are frozen from the start.
__global__ void k_bctrl_inner(BatchCtrl* in, const BatchCtrl* out, double eta, int max_iter,
                              int Kc) {
  in->c = Ctrl{};
  in->c.max_iter = max_iter;
  int all = 1;
  for (int k = 0; k < kMaxK; ++k) {
    const int dn = k < Kc ? out->kdone[k] : 1;
    in->kdone[k] = dn;
    in->kiter[k] = 0;
    in->kstatus[k] = PSI_OK;
    in->kgap[k] = 0.0;
    in->ktol[k] = fmax(eta * out->kgap[k], 0.5 * out->ktol[k]);
    all &= dn;
  }
  in->c.done = all;
}

// ---------------------------------------------------------------- origins
__global__ void k_bzero(double* a, double* b, int64_t total) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= total) return;
  a[t] = 0.0;
  b[t] = 0.0;
}

// Σ_j c_j P[j, k] per workgroup in row order (optionally copying P to the
// caller's [N × K] output at column k0 + k).
__global__ __launch_bounds__(kBlock) void k_origin_colsum(const double* P, const double* c,
                                                         int64_t n, int Kc, int K, int k0,
                                                         double* p_out, double* part) {
  __shared__ double red[kBlock / 64][kMaxK];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int k = lane < Kc ? lane : Kc - 1;
  double acc = 0.0;
  for (int64_t r = int64_t(blockIdx.x) * (kBlock / 64) + wave; r < n;
       r += int64_t(gridDim.x) * (kBlock / 64)) {
    const double v = P[r * Kc + k];
    acc += c[r] * v;
    if (p_out && lane < Kc) p_out[r * K + k0 + lane] = v;
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && lane < Kc)
    part[int64_t(blockIdx.x) * Kc + lane] =
        ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// ψ_i = (Σ_j c_j p_i^(j) + d_i) / N, the workgroup partials in order.
__global__ void k_origin_psi(const double* part, int n_blk, int Kc, const int* origin,
                             const double* d, double inv_n, double* psi_out) {
  const int k = threadIdx.x;
  if (k >= Kc) return;
  double sum = 0.0;
  for (int b = 0; b < n_blk; ++b) sum += part[int64_t(b) * Kc + k];
  psi_out[k] = (sum + d[origin[k]]) * inv_n;
}

// ---------------------------------------------------------------- graphs
// Per-graph gap of a block-diagonal operator: graph g sums its users' |Δ| in
// a fixed order, records it, and freezes when it meets the tolerance (a graph
// frozen before this pass was copied into both buffers by it, so it is marked
// skippable); the last graph to report sets done when every graph is done.
// One counter carries both the arrivals (low 16 bits) and the done graphs
// (high bits).
__global__ __launch_bounds__(kGraphGapBlock) void k_graph_gap(const int64_t* graph_off,
                                                              int n_graphs,
                                                              const double* row_delta, Ctrl* ctrl,
                                                              int* gdone, int* gskip, int* giter,
                                                              int* gstatus, double* ggap,
                                                              const double* gtol) {
  constexpr int W = kGraphGapBlock / 64;
  __shared__ double red[W];
  if (ctrl->done) return;
  const int g = blockIdx.x;
  const int was_done = gdone[g];
  double sum = 0.0;
  if (!was_done) {
    // thread t adds users t, t + B, t + 2B, ... of the graph in order, eight loads in flight
    const int64_t r1 = graph_off[g + 1];
    int64_t r = graph_off[g] + threadIdx.x;
    for (; r + 7 * kGraphGapBlock < r1; r += 8 * kGraphGapBlock) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = row_delta[r + u * kGraphGapBlock];
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += v[u];
    }
    for (; r < r1; r += kGraphGapBlock) sum += row_delta[r];
  }
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x != 0) return;
  int done = was_done;
  // a graph frozen before this pass was copied into both buffers by it
  if (was_done) gskip[g] = 1;
  if (!was_done) {
    double G = 0.0;
    for (int w = 0; w < W; ++w) G += red[w];
    const int it = giter[g] + 1;
    giter[g] = it;
    ggap[g] = G;
    if (!isfinite(G)) {
      done = 1;
      gstatus[g] = PSI_ENUMERIC;
    } else if (G <= (gtol ? gtol[g] : ctrl->tol)) {
      done = 1;
      gstatus[g] = PSI_OK;
    } else if (it >= ctrl->max_iter) {
      done = 1;
      gstatus[g] = PSI_ENOTCONV;
    }
    gdone[g] = done;
  }
  const unsigned t = atomicAdd(&ctrl->ticket, 1u + (static_cast<unsigned>(done) << 16));
  if ((t & 0xFFFFu) == static_cast<unsigned>(n_graphs) - 1u) {
    const unsigned n_done = (t >> 16) + static_cast<unsigned>(done);
    ctrl->ticket = 0;
    ctrl->iter += 1;
    if (n_done == static_cast<unsigned>(n_graphs)) publish_done(ctrl, -1);
  }
}

__global__ void k_graph_init(const double* c, const double* invden, int64_t n, int n_graphs,
                             double* s, double* z, int* gdone, int* gskip, int* giter,
                             int* gstatus, double* ggap, Ctrl* ctrl, double tol, int max_iter) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    s[i] = c[i];
    z[i] = invden[i] * c[i];
  }
  if (i < n_graphs) {
    gdone[i] = 0;
    gskip[i] = 0;
    giter[i] = 0;
    gstatus[i] = PSI_OK;
    ggap[i] = 0.0;
  }
  if (i == 0) {
    // a pending wait time-out and the host's test switch survive the reset
    const unsigned err = ctrl->err_flags;
    const int force = ctrl->force_timeout;
    *ctrl = Ctrl{};
    ctrl->err_flags = err;
    ctrl->force_timeout = force;
    ctrl->tol = tol;
    ctrl->max_iter = max_iter;
    ctrl->bnorm = 1.0;
  }
}

// Per-graph state of an iteration reset (every graph live), with its control
// block: a pending wait time-out and the host's test switch survive.
__global__ void k_graph_reset(int n_graphs, int* gdone, int* gskip, int* giter, int* gstatus,
                              double* ggap, Ctrl* ctrl, double tol, int max_iter) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n_graphs) {
    gdone[g] = 0;
    gskip[g] = 0;
    giter[g] = 0;
    gstatus[g] = PSI_OK;
    ggap[g] = 0.0;
  }
  if (g == 0) {
    const unsigned err = ctrl->err_flags;
    const int force = ctrl->force_timeout;
    *ctrl = Ctrl{};
    ctrl->err_flags = err;
    ctrl->force_timeout = force;
    ctrl->tol = tol;
    ctrl->max_iter = max_iter;
    ctrl->bnorm = 1.0;
  }
}

// The correction solves of a mixed-precision graph batch: graph g runs to
// eta·‖r_g‖₁ (its last FP64 gap), or to half the batch's L1 tolerance when
// that is larger; graphs already finished are frozen from the start.
__global__ void k_graph_inner_init(int n_graphs, const int* gdone, const double* ggap, double eta,
                                   double tol, int* gdone2, int* gskip2, int* giter2,
                                   int* gstatus2, double* ggap2, double* gtol, Ctrl* ctrl2,
                                   int max_iter) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n_graphs) {
    gdone2[g] = gdone[g];
    gskip2[g] = 0;
    giter2[g] = 0;
    gstatus2[g] = PSI_OK;
    ggap2[g] = 0.0;
    gtol[g] = fmax(eta * ggap[g], 0.5 * tol);
  }
  if (g == 0) {
    const unsigned err = ctrl2->err_flags;
    const int force = ctrl2->force_timeout;
    *ctrl2 = Ctrl{};
    ctrl2->err_flags = err;
    ctrl2->force_timeout = force;
    ctrl2->tol = 0.0;
    ctrl2->max_iter = max_iter;
    ctrl2->bnorm = 1.0;
  }
}

// r = Y − X rounded to FP32 (the FP64 residual of X); e_0 = r, z_e = e/den.
__global__ void k_graph_prep_inner(const double* Y, const double* X, const float* invden32,
                                   int64_t n, float* r32, float* e, float* ze) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float r = static_cast<float>(Y[i] - X[i]);
  r32[i] = r;
  e[i] = r;
  ze[i] = invden32[i] * r;
}

// After a correction solve: X ← X + e in the graphs still running; a graph
// that has finished takes its final step Y.
__global__ void k_graph_update(double* X, double* zX, const double* Y, const double* zY,
                               const float* e, const double* invden, const int* graph_of,
                               const int* gdone, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (gdone[graph_of[i]]) {
    X[i] = Y[i];
    zX[i] = zY[i];
  } else {
    const double v = X[i] + static_cast<double>(e[i]);
    X[i] = v;
    zX[i] = invden[i] * v;
  }
}

// Hub-finishing grid: four hubs per workgroup, at most kHubFinGrid workgroups.
int hub_finish_grid(int64_t n_hubs, int G) {
  const int64_t per = 4 * int64_t(G);
  return static_cast<int>(
      std::max<int64_t>(1, std::min<int64_t>(kHubFinGrid, (n_hubs + per - 1) / per)));
}

// Lane groups of a tile of Kc scenarios: as many as fit a wave.
int lane_groups(int Kc) { return Kc <= 8 ? 8 : Kc <= 16 ? 4 : Kc <= 32 ? 2 : 1; }

template <int BM, int G>
void launch_spmm_g(const BArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_spmm_rows<BM, G>), dim3(grid), dim3(kBlock), 0, st, a);
  if (a.n_chunks)
    hipLaunchKernelGGL((k_spmm_hub_chunk<BM, G>), dim3((a.n_chunks + G - 1) / G), dim3(kBlock), 0,
                       st, a);
  if (a.n_hubs)
    hipLaunchKernelGGL((k_spmm_hub_finish<BM, G>), dim3(hub_finish_grid(a.n_hubs, G)),
                       dim3(kBlock), 0, st, a);
}

// One multi-vector product of mode BM: the rows kernel (grid workgroups),
// then the hub chunks and the hub rows.
template <int BM>
void launch_spmm(const BArgs& a, int grid, hipStream_t st) {
  switch (lane_groups(a.Kc)) {
    case 8: return launch_spmm_g<BM, 8>(a, grid, st);
    case 4: return launch_spmm_g<BM, 4>(a, grid, st);
    case 2: return launch_spmm_g<BM, 2>(a, grid, st);
    default: return launch_spmm_g<BM, 1>(a, grid, st);
  }
}

// Workgroups of the hub-finishing kernel of a product (its gap partials).
int hub_blocks(const BArgs& a) {
  return a.n_hubs ? hub_finish_grid(a.n_hubs, lane_groups(a.Kc)) : 0;
}

// The gap of a pass: kGapParts first-level sums of the n_blk rows-kernel and
// n_hblk hub-kernel partials, then one wave decides.
void launch_batch_gap(const BArgs& a, int n_blk, int n_hblk, hipStream_t st) {
  hipLaunchKernelGGL(k_batch_gap_part, dim3(kGapParts), dim3(kBlock), 0, st, a, n_blk, n_hblk);
  hipLaunchKernelGGL(k_batch_gap, dim3(1), dim3(64), 0, st, a);
}

int rows_grid() {
  static int cap = 0;
  if (!cap) {
    int dev = 0, per_cu = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmm_rows<kScen, 1>, kBlock, 0);
    cap = std::min(kMaxGrid, std::max(1, per_cu) * std::max(1, cus));
  }
  return cap;
}

}  // namespace

// Row tiles, hub rows and hub chunks of the pattern `row_ptr` (n rows, m
// entries); blocks to learn the hub and chunk counts.
struct BSched {
  uint32_t n_hubs = 0, n_chunks = 0;
  int64_t n_wtiles = 0;
};

static psi_status batch_schedule(const int* row_ptr, int64_t n, int64_t m, BatchWs& w,
                                 int items, int chunk_edges, hipStream_t st, BSched* out) {
  // hub rows and their chunks (depend only on the pattern)
  hipLaunchKernelGGL(k_hub_flags, dim3(grid_for(n + 1)), dim3(kBlock), 0, st, row_ptr, n,
                     w.flags);
  psi_status s = scan_exclusive_u32(w.flags, w.flags, n + 1, w.scan_tmp,
                                    w.scan_tmp + scan_tile_count(n + 1) + 4, st);
  if (s != PSI_OK) return s;
  uint32_t n_hubs = 0;
  PSI_HIP_CHECK(hipMemcpyAsync(&n_hubs, w.flags + n, 4, hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  uint32_t* nchunks = reinterpret_cast<uint32_t*>(w.chunk_row);  // counts, then scanned in place
  uint32_t n_chunks = 0;
  if (n_hubs > 0) {
    hipLaunchKernelGGL(k_hub_list, dim3(grid_for(n)), dim3(kBlock), 0, st, row_ptr, n,
                       w.flags, chunk_edges, w.hub_rows, nchunks);
    uint32_t* chunk0 = reinterpret_cast<uint32_t*>(w.chunk_e0);
    PSI_HIP_CHECK(hipMemsetAsync(nchunks + n_hubs, 0, 4, st));
    s = scan_exclusive_u32(nchunks, chunk0, int64_t(n_hubs) + 1, w.scan_tmp,
                           w.scan_tmp + scan_tile_count(n + 1) + 4, st);
    if (s != PSI_OK) return s;
    PSI_HIP_CHECK(hipMemcpyAsync(&n_chunks, chunk0 + n_hubs, 4, hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    // hub_chunk0 = chunk0 (copied), then the chunk table overwrites the scratch
    PSI_HIP_CHECK(hipMemcpyAsync(w.hub_chunk0, chunk0, 4 * size_t(n_hubs + 1),
                                 hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_chunk_table, dim3(grid_for(n_hubs)), dim3(kBlock), 0, st, row_ptr,
                       w.hub_rows, reinterpret_cast<const uint32_t*>(w.hub_chunk0), int(n_hubs),
                       chunk_edges, w.chunk_row, w.chunk_e0, w.hub_chunk0);
  }
  const int64_t n_wtiles = std::max<int64_t>((n + m + items - 1) / items, 1);
  hipLaunchKernelGGL(k_row_tiles, dim3(grid_for(n_wtiles + 1)), dim3(kBlock), 0, st, row_ptr,
                     n, m, int64_t(items), n_wtiles, w.row_tiles);
  PSI_HIP_CHECK(hipGetLastError());

  out->n_hubs = n_hubs;
  out->n_chunks = n_chunks;
  out->n_wtiles = n_wtiles;
  return PSI_OK;
}

// Pass arguments of a scenario tile of Kc scenarios (the tile's data in w).
static BArgs scenario_args(const psi_operator* op, const BatchWs& w, const BSched& sc, int Kc,
                           int chunk) {
  BArgs b{};
  b.row_ptr = op->row_ptr;
  b.col = op->col;
  b.n_rows = static_cast<int>(op->n);
  b.Kc = Kc;
  b.row_tiles = w.row_tiles;
  b.n_wtiles = static_cast<int>(sc.n_wtiles);
  b.hub_rows = w.hub_rows;
  b.hub_chunk0 = w.hub_chunk0;
  b.n_hubs = static_cast<int>(sc.n_hubs);
  b.chunk_row = w.chunk_row;
  b.chunk_e0 = w.chunk_e0;
  b.n_chunks = static_cast<int>(sc.n_chunks);
  b.chunk_edges = chunk;
  b.c = w.c;
  b.mu = w.mu;
  b.invden = w.invden;
  b.lam = w.lam;
  b.d = w.d;
  b.inv_n = 1.0 / static_cast<double>(op->n);
  b.chunk_part = w.chunk_part;
  b.gap_blk = w.gap_blk;
  b.gap_hub = w.gap_hub;
  b.gap_lvl = w.gap_lvl;
  b.ctrl = w.ctrl;
  b.r32 = w.r32;
  b.mu32 = w.mu32;
  b.invden32 = w.invden32;
  return b;
}

psi_status batched_workspace_size(const psi_operator* op, int n_scenarios, int precision,
                                  size_t* bytes) {
  PSI_REQUIRE(bytes, "bytes must not be NULL");
  PSI_REQUIRE(n_scenarios >= 1, "n_scenarios must be >= 1");
  PSI_REQUIRE(precision == PSI_PREC_FP64 || precision == PSI_PREC_MIXED,
              "batched solves run in PSI_PREC_FP64 or PSI_PREC_MIXED");
  *bytes = batch_layout(op->n, op->m, nullptr, nullptr, precision == PSI_PREC_MIXED);
  return PSI_OK;
}

psi_status solve_batched(psi_operator* op, const psi_params* prm, int K, const double* lam_in,
                         const double* mu_in, double* psi_out, psi_info* infos, void* ws,
                         size_t ws_bytes, hipStream_t st) {
  PSI_REQUIRE(prm && psi_out && ws, "params, psi_out and workspace must not be NULL");
  PSI_REQUIRE(lam_in && mu_in, "lambda and mu must not be NULL in scenario mode");
  PSI_REQUIRE(K >= 1, "n_scenarios must be >= 1");
  PSI_REQUIRE(prm->tol > 0.0 && std::isfinite(prm->tol), "tol must be finite and > 0");
  PSI_REQUIRE(prm->max_iter > 0, "max_iter must be > 0");
  PSI_REQUIRE(prm->tol_mode == PSI_TOL_ABS_L1, "batched solves use PSI_TOL_ABS_L1");
  PSI_REQUIRE(prm->precision == PSI_PREC_FP64 || prm->precision == PSI_PREC_MIXED,
              "batched solves run in PSI_PREC_FP64 or PSI_PREC_MIXED");
  PSI_REQUIRE(op->n_graphs == 1, "scenario batches need a single-graph operator");
  const bool mixed = prm->precision == PSI_PREC_MIXED;
  size_t need = batch_layout(op->n, op->m, nullptr, nullptr, mixed);
  if (ws_bytes < need) {
    set_error("batched workspace smaller than psi_batched_workspace_size reported");
    return PSI_ENOSPACE;
  }
  // the schedule: explicit, else tuned for this precision, else the defaults
  const int pi = prm->precision;
  const int Kt = prm->batch_tile ? prm->batch_tile
                                 : (op->tuned_batch_tile[pi] ? op->tuned_batch_tile[pi] : kMaxK);
  const int items = prm->batch_items ? prm->batch_items
                                     : (op->tuned_batch_items[pi] ? op->tuned_batch_items[pi]
                                                                  : kWaveItems);
  const int chunk = prm->hub_chunk ? prm->hub_chunk
                                   : (op->tuned_batch_chunk[pi] ? op->tuned_batch_chunk[pi]
                                                                : kChunkEdges);
  PSI_REQUIRE(Kt >= 1 && Kt <= kMaxK, "batch_tile must be 0 or in [1, 64]");
  PSI_REQUIRE(items >= kMinWaveItems && items <= 8192, "batch_items must be 0 or in [128, 8192]");
  PSI_REQUIRE(chunk >= kMinChunkEdges && chunk <= kMaxChunkEdges,
              "hub_chunk must be 0 or in [512, 8192]");
  BatchWs w{};
  batch_layout(op->n, op->m, &w, static_cast<char*>(ws), mixed);
  const int64_t n = op->n, m = op->m;

  BSched sc{};
  psi_status s = batch_schedule(op->row_ptr, n, m, w, items, chunk, st, &sc);
  if (s != PSI_OK) return s;
  const uint32_t n_hubs = sc.n_hubs, n_chunks = sc.n_chunks;
  const int64_t n_wtiles = sc.n_wtiles;

  struct Pinned {
    BatchCtrl* p = nullptr;
    ~Pinned() {
      if (p) (void)hipHostFree(p);
    }
  } pinned;
  PSI_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&pinned.p), 2 * sizeof(BatchCtrl),
                              hipHostMallocDefault));
  BatchCtrl* h = pinned.p;       // the scenarios' own iteration
  BatchCtrl* h2 = pinned.p + 1;  // a correction solve
  const int grid = std::min(rows_grid(), static_cast<int>(n_wtiles));
  const double eta = prm->inner_tol > 0.0 ? prm->inner_tol : 2e-6;
  EventPair evp;
  PSI_HIP_CHECK(hipEventCreate(&evp.a));
  PSI_HIP_CHECK(hipEventCreate(&evp.b));
  hipEvent_t ev0 = evp.a, ev1 = evp.b;
  PSI_HIP_CHECK(hipEventRecord(ev0, st));
  int worst = PSI_OK;
  for (int k0 = 0; k0 < K; k0 += Kt) {
    const int Kc = std::min(Kt, K - k0);
    const int64_t nk = n * Kc;
    hipLaunchKernelGGL(k_bctrl_init, dim3(1), dim3(1), 0, st, w.ctrl, prm->tol, prm->max_iter);
    hipLaunchKernelGGL(k_bprep_act, dim3(grid_for(nk)), dim3(kBlock), 0, st, lam_in, mu_in, n, K,
                       k0, Kc, w.lam, w.mu, &w.ctrl->c);
    hipLaunchKernelGGL(k_bprep_den, dim3(grid_for(n * 64)), dim3(kBlock), 0, st, op->fm_row_ptr,
                       op->fm_col, w.lam, w.mu, n, Kc, w.invden, w.c, w.d);
    hipLaunchKernelGGL(k_binit, dim3(grid_for(nk)), dim3(kBlock), 0, st, w.c, w.invden, nk, w.s_a,
                       w.z_a);
    if (mixed)
      hipLaunchKernelGGL(k_bprep32, dim3(grid_for(nk)), dim3(kBlock), 0, st, w.mu, w.invden, nk,
                         w.mu32, w.invden32);
    PSI_HIP_CHECK(hipGetLastError());
    const BArgs base = scenario_args(op, w, sc, Kc, chunk);
    // one FP64 step s_new = Aᵀ s_old + c of every scenario (z = s / den
    // gathered), or the final ψ pass from z
    auto pass64 = [&](const double* z, const double* s_old, double* s_new, double* z_new,
                      bool final_pass) -> psi_status {
      BArgs a = base;
      a.z = z;
      a.s_old = s_old;
      a.s_new = s_new;
      a.z_new = z_new;
      if (final_pass) {
        a.psi = psi_out;
        a.psi_ld = K;
        a.psi_col0 = k0;
        launch_spmm<kScenFinal>(a, grid, st);
      } else {
        launch_spmm<kScen>(a, grid, st);
        launch_batch_gap(a, grid, hub_blocks(a), st);
      }
      PSI_HIP_CHECK(hipGetLastError());
      return PSI_OK;
    };
    // step i of a correction solve e = Aᵀe + r (FP32, buffers alternate)
    auto pass32 = [&](int i) -> psi_status {
      BArgs a = base;
      const bool even = (i & 1) == 0;
      a.ctrl = w.ctrl2;
      a.z32 = even ? w.ze_a : w.ze_b;
      a.e_old = even ? w.e_a : w.e_b;
      a.e_new = even ? w.e_b : w.e_a;
      a.ze_new = even ? w.ze_b : w.ze_a;
      launch_spmm<kScen32>(a, grid, st);
      launch_batch_gap(a, grid, hub_blocks(a), st);
      PSI_HIP_CHECK(hipGetLastError());
      return PSI_OK;
    };
    // enqueue steps in blocks (growing unless check_every is set) and read the
    // control block between blocks; steps after the last scenario finished
    // exit at once
    auto loop = [&](BatchCtrl* dctrl, BatchCtrl* hctrl, int budget, auto&& step) -> psi_status {
      int enq = 0, chunk = prm->check_every > 0 ? prm->check_every : 8;
      while (true) {
        const int cnt = std::min(chunk, budget - enq);
        for (int i = 0; i < cnt; ++i) {
          psi_status r = step(enq + i);
          if (r != PSI_OK) return r;
        }
        enq += cnt;
        PSI_HIP_CHECK(hipMemcpyAsync(hctrl, dctrl, sizeof(BatchCtrl), hipMemcpyDeviceToHost, st));
        PSI_HIP_CHECK(hipStreamSynchronize(st));
        if (hctrl->c.err_flags & kErrActivity) {
          set_error("activity must satisfy lambda > 0 and mu >= 0, both finite");
          return PSI_EINVAL;
        }
        if (hctrl->c.done || enq >= budget) break;
        if (prm->check_every == 0) chunk = std::min(2 * chunk, 64);
      }
      return PSI_OK;
    };
    // plain FP64 steps from (P, zP), the other buffer pair (Q, zQ) taking
    // turns, after `before` steps of this tile; returns the pair that holds
    // the last step
    auto plain = [&](double* P, double* zP, double* Q, double* zQ, int budget, int before,
                     const double** z_last) -> psi_status {
      psi_status r = loop(w.ctrl, h, budget, [&](int i) {
        const bool even = (i & 1) == 0;
        return pass64(even ? zP : zQ, even ? P : Q, even ? Q : P, even ? zQ : zP, false);
      });
      if (r != PSI_OK) return r;
      *z_last = ((h->c.iter - before) & 1) ? zQ : zP;
      return PSI_OK;
    };
    std::vector<int> fp32_passes(Kc, 0), refinements(Kc, 0);
    const double* z_fin = nullptr;
    if (!mixed) {
      s = plain(w.s_a, w.z_a, w.s_b, w.z_b, prm->max_iter, 0, &z_fin);
      if (s != PSI_OK) return s;
    } else {
      double *X = w.s_a, *zX = w.z_a, *Y = w.s_b, *zY = w.z_b;
      std::vector<double> prev(Kc, std::numeric_limits<double>::infinity());
      while (true) {
        // FP64 residual pass: Y = Aᵀ X + c, gap_k = ‖Y_k − X_k‖₁
        s = pass64(zX, X, Y, zY, false);
        if (s != PSI_OK) return s;
        PSI_HIP_CHECK(hipMemcpyAsync(h, w.ctrl, sizeof(BatchCtrl), hipMemcpyDeviceToHost, st));
        PSI_HIP_CHECK(hipStreamSynchronize(st));
        if (h->c.err_flags & kErrActivity) {
          set_error("activity must satisfy lambda > 0 and mu >= 0, both finite");
          return PSI_EINVAL;
        }
        z_fin = zY;
        if (h->c.done) break;
        bool gains = true;
        for (int k = 0; k < Kc; ++k)
          if (!h->kdone[k] && !(h->kgap[k] < 0.25 * prev[k])) gains = false;
        if (!gains) {
          // a refinement no longer gains for some scenario: plain FP64 steps from Y
          s = plain(Y, zY, X, zX, std::max(1, prm->max_iter - h->c.iter), h->c.iter, &z_fin);
          if (s != PSI_OK) return s;
          break;
        }
        for (int k = 0; k < Kc; ++k) {
          prev[k] = h->kgap[k];
          if (!h->kdone[k]) ++refinements[k];
        }
        // FP32 correction solve e = Aᵀe + r, each scenario to η‖r‖₁
        hipLaunchKernelGGL(k_bprep_inner, dim3(grid_for(nk)), dim3(kBlock), 0, st, Y, X,
                           w.invden32, nk, w.r32, w.e_a, w.ze_a);
        hipLaunchKernelGGL(k_bctrl_inner, dim3(1), dim3(1), 0, st, w.ctrl2, w.ctrl, eta,
                           prm->max_iter, Kc);
        PSI_HIP_CHECK(hipGetLastError());
        s = loop(w.ctrl2, h2, prm->max_iter, pass32);
        if (s != PSI_OK) return s;
        for (int k = 0; k < Kc; ++k) fp32_passes[k] += h2->kiter[k];
        const float* e_fin = (h2->c.iter & 1) ? w.e_b : w.e_a;
        hipLaunchKernelGGL(k_bupdate, dim3(grid_for(nk)), dim3(kBlock), 0, st, X, zX, Y, zY,
                           e_fin, w.invden, w.ctrl, nk, Kc);
        PSI_HIP_CHECK(hipGetLastError());
      }
    }
    s = pass64(z_fin, nullptr, nullptr, nullptr, true);
    if (s != PSI_OK) return s;
    for (int k = 0; k < Kc; ++k) {
      int stk = h->kdone[k] ? h->kstatus[k] : PSI_ENOTCONV;
      if (stk != PSI_OK && worst == PSI_OK) worst = stk;
      if (infos) {
        psi_info& inf = infos[k0 + k];
        inf = psi_info{};
        inf.status = stk;
        inf.iterations = h->kiter[k];
        inf.fp32_passes = fp32_passes[k];
        inf.refinements = refinements[k];
        inf.spmv_passes = h->kiter[k] + fp32_passes[k] + 1;
        inf.final_gap = h->kgap[k];
        inf.final_l1_step = h->kgap[k];
        inf.col_segments = 1;
        inf.tile_items = items;
        inf.batch_tile = Kt;
        inf.hub_chunk = chunk;
      }
    }
  }
  PSI_HIP_CHECK(hipEventRecord(ev1, st));
  PSI_HIP_CHECK(hipEventSynchronize(ev1));
  float ms = 0.f;
  PSI_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
  if (infos)
    for (int k = 0; k < K; ++k) infos[k].device_ms = ms;
  if (worst != PSI_OK) set_error("a scenario did not converge (see its info)");
  return static_cast<psi_status>(worst);
}

// The schedule of a graph batch in `precision`: explicit, else tuned, else by
// default batches of at least 10^6 users take two segments with tiled partial
// passes: the graphs lie in one segment or the other, and the partial kernel
// plus a streaming combine beat the fused pass with its per-graph epilogue
// (measured on 256 graphs of 13.3M users: 84 against 96 ms).
static psi_status graph_schedule(psi_operator* op, const psi_params* prm, int precision,
                                 int* tile, int* S, int* form) {
  const bool tuned = op->tuned_graph_S[precision] > 0;
  *tile = prm->tile_items ? prm->tile_items
        : tuned           ? op->tuned_graph_tile[precision]
        : (op->sched_items ? op->sched_items : kDefaultTileItems);
  PSI_REQUIRE(tile_items_supported(*tile), "unsupported tile_items");
  const bool big = op->n >= 1000000;
  *S = prm->col_segments ? prm->col_segments : tuned ? op->tuned_graph_S[precision] : (big ? 2 : 1);
  PSI_REQUIRE(*S == 1 || *S == 2 || *S == 4 || *S == 8, "col_segments must be 0, 1, 2, 4 or 8");
  PSI_REQUIRE(precision != PSI_PREC_MIXED || *S <= 4,
              "a mixed-precision graph batch takes at most 4 column segments");
  PSI_REQUIRE(prm->seg_form != PSI_SEG_BANDS && prm->seg_form != PSI_SEG_BINS,
              "graph batches have no band or binned layout");
  const int req = prm->seg_form ? prm->seg_form
                : (tuned && !prm->col_segments) ? op->tuned_graph_form[precision]
                : (big && *S > 1 ? kSegTiles : 0);
  return resolve_form(op, req, *S, precision, *S, precision == PSI_PREC_MIXED ? 4 : 8, form);
}

// One step pass of a graph batch: the FP64 step X → Y (outer state) or an
// FP32 correction step e_i → e_{i+1} (inner state), then the per-graph gaps.
// `skip`: gathers of graphs frozen a whole pass are skipped.
static psi_status graph_pass(psi_operator* op, int S, bool fp32, int i, const double* X,
                             const double* zX, double* Y, double* zY, Ctrl* ctrl, bool skip,
                             const double* gtol, hipStream_t st) {
  const int G = op->n_graphs;
  const int off = fp32 ? G : 0;
  PassArgs a = base_args(op);
  a.count_iter = 0;
  a.respect_done = 1;
  a.ctrl = ctrl;
  a.gdone = op->gdone + off;
  a.gskip = skip ? op->gskip + off : nullptr;
  if (fp32) {
    const bool even = (i & 1) == 0;
    a.x = even ? op->ze_a : op->ze_b;
    a.e_old = even ? op->e_a : op->e_b;
    a.e_new = even ? op->e_b : op->e_a;
    a.ze_new = even ? op->ze_b : op->ze_a;
    a.r32 = op->r32;
  } else {
    a.x = zX;
    a.s_old = X;
    a.s_new = Y;
    a.z_new = zY;
  }
  const PassMode mode = fp32 ? kStep32G : kStep64G;
  psi_status r = S > 1 ? launch_pass_seg(op, mode, a, st) : launch_pass(op, mode, a, st);
  if (r != PSI_OK) return r;
  hipLaunchKernelGGL(k_graph_gap, dim3(G), dim3(kGraphGapBlock), 0, st, op->graph_off, G,
                     op->row_delta, ctrl, op->gdone + off, op->gskip + off, op->giter + off,
                     op->gstatus + off, op->ggap + off, gtol);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

// A graph batch to its tolerance; psi_out may be NULL (no final ψ pass: the
// autotuner's timing runs), *ms_out (if given) the device time of the solve.
static psi_status graph_solve(psi_operator* op, const psi_params* prm, double* psi_out,
                              psi_info* infos, hipStream_t st, float* ms_out) {
  PSI_REQUIRE(prm, "params must not be NULL");
  PSI_REQUIRE(op->n_graphs > 1, "graph mode needs a multi-graph operator");
  PSI_REQUIRE(prm->tol > 0.0 && std::isfinite(prm->tol), "tol must be finite and > 0");
  PSI_REQUIRE(prm->max_iter > 0, "max_iter must be > 0");
  PSI_REQUIRE(prm->tol_mode == PSI_TOL_ABS_L1, "graph batches use PSI_TOL_ABS_L1");
  PSI_REQUIRE(prm->precision == PSI_PREC_FP64 || prm->precision == PSI_PREC_MIXED,
              "graph batches run in PSI_PREC_FP64 or PSI_PREC_MIXED");
  const bool mixed = prm->precision == PSI_PREC_MIXED;
  int tile = 0, S = 1, form = 0;
  psi_status s = graph_schedule(op, prm, prm->precision, &tile, &S, &form);
  if (s != PSI_OK) return s;
  s = prepare(op, tile, S, form, st);
  if (s != PSI_OK) return s;
  const int64_t n = op->n;
  const int G = op->n_graphs;
  EventPair evp;
  PSI_HIP_CHECK(hipEventCreate(&evp.a));
  PSI_HIP_CHECK(hipEventCreate(&evp.b));
  hipEvent_t ev0 = evp.a, ev1 = evp.b;
  PSI_HIP_CHECK(hipEventRecord(ev0, st));
  hipLaunchKernelGGL(k_graph_init, dim3(grid_for(std::max<int64_t>(n, G))), dim3(kBlock), 0, st,
                     op->c, op->invden, n, G, op->s_a, op->z_a, op->gdone, op->gskip, op->giter,
                     op->gstatus, op->ggap, op->ctrl, prm->tol, prm->max_iter);
  Ctrl* h = op->host_ctrl;
  // enqueue passes in blocks (growing unless check_every is set) and read the
  // control block between blocks; passes after the last graph finished exit
  // at once.  Returns the number of passes enqueued.
  auto loop = [&](Ctrl* dctrl, int budget, auto&& pass, int* enqueued) -> psi_status {
    int enq = 0, chunk = prm->check_every > 0 ? prm->check_every : 8;
    while (true) {
      const int cnt = std::min(chunk, budget - enq);
      for (int i = 0; i < cnt; ++i) {
        psi_status r = pass(enq + i);
        if (r != PSI_OK) return r;
      }
      enq += cnt;
      PSI_HIP_CHECK(hipMemcpyAsync(h, dctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
      PSI_HIP_CHECK(hipStreamSynchronize(st));
      if (h->err_flags & kErrSlotTimeout) return check_waits(op, st);
      if (h->done || enq >= budget) break;
      if (prm->check_every == 0) chunk = std::min(2 * chunk, 64);
    }
    *enqueued = enq;
    return PSI_OK;
  };
  // plain FP64 steps from (P, zP), (Q, zQ) taking turns; returns the z of the
  // buffer that holds the last step in *z_last
  auto plain = [&](double* P, double* zP, double* Q, double* zQ, int budget,
                   const double** z_last) -> psi_status {
    const int before = 0;
    (void)before;
    Ctrl* c0 = op->ctrl;
    int it0 = 0;
    PSI_HIP_CHECK(hipMemcpyAsync(h, c0, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    it0 = h->iter;
    int enq = 0;
    psi_status r = loop(c0, budget, [&](int i) {
      const bool even = (i & 1) == 0;
      return graph_pass(op, S, false, i, even ? P : Q, even ? zP : zQ, even ? Q : P,
                        even ? zQ : zP, c0, true, nullptr, st);
    }, &enq);
    if (r != PSI_OK) return r;
    *z_last = ((h->iter - it0) & 1) ? zQ : zP;
    return PSI_OK;
  };
  std::vector<int> fp32(G, 0), refine(G, 0);
  const double* z_fin = nullptr;
  if (!mixed) {
    s = plain(op->s_a, op->z_a, op->s_b, op->z_b, prm->max_iter, &z_fin);
    if (s != PSI_OK) return s;
  } else {
    // FP64 residual passes X → Y, each followed by FP32 correction solves of
    // the graphs still running, X ← X + e (as the single-graph mixed solve)
    const double eta = prm->inner_tol > 0.0 ? prm->inner_tol : 2e-6;
    double *X = op->s_a, *zX = op->z_a, *Y = op->s_b, *zY = op->z_b;
    std::vector<double> prev(G, std::numeric_limits<double>::infinity()), gap(G);
    std::vector<int> dn(G), it2(G);
    while (true) {
      s = graph_pass(op, S, false, 0, X, zX, Y, zY, op->ctrl, true, nullptr, st);
      if (s != PSI_OK) return s;
      PSI_HIP_CHECK(hipMemcpyAsync(h, op->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
      PSI_HIP_CHECK(hipMemcpyAsync(gap.data(), op->ggap, 8 * size_t(G), hipMemcpyDeviceToHost, st));
      PSI_HIP_CHECK(hipMemcpyAsync(dn.data(), op->gdone, 4 * size_t(G), hipMemcpyDeviceToHost, st));
      PSI_HIP_CHECK(hipStreamSynchronize(st));
      if (h->err_flags & kErrSlotTimeout) return check_waits(op, st);
      z_fin = zY;
      if (h->done || h->iter >= prm->max_iter) break;
      bool gains = true;
      for (int g = 0; g < G; ++g)
        if (!dn[g] && !(gap[g] < 0.25 * prev[g])) gains = false;
      if (!gains) {
        // a refinement no longer gains for some graph: plain FP64 steps from Y
        s = plain(Y, zY, X, zX, std::max(1, prm->max_iter - h->iter), &z_fin);
        if (s != PSI_OK) return s;
        break;
      }
      for (int g = 0; g < G; ++g) {
        prev[g] = gap[g];
        if (!dn[g]) ++refine[g];
      }
      hipLaunchKernelGGL(k_graph_prep_inner, dim3(grid_for(n)), dim3(kBlock), 0, st, Y, X,
                         op->invden32, n, op->r32, op->e_a, op->ze_a);
      hipLaunchKernelGGL(k_graph_inner_init, dim3(grid_for(G)), dim3(kBlock), 0, st, G,
                         op->gdone, op->ggap, eta, prm->tol, op->gdone + G, op->gskip + G,
                         op->giter + G, op->gstatus + G, op->ggap + G, op->gtol, op->ctrl + 1,
                         prm->max_iter);
      PSI_HIP_CHECK(hipGetLastError());
      int enq = 0;
      s = loop(op->ctrl + 1, prm->max_iter, [&](int i) {
        return graph_pass(op, S, true, i, nullptr, nullptr, nullptr, nullptr, op->ctrl + 1, true,
                          op->gtol, st);
      }, &enq);
      if (s != PSI_OK) return s;
      const int inner_passes = h->iter;  // h holds the inner control block
      PSI_HIP_CHECK(hipMemcpyAsync(it2.data(), op->giter + G, 4 * size_t(G),
                                   hipMemcpyDeviceToHost, st));
      PSI_HIP_CHECK(hipStreamSynchronize(st));
      for (int g = 0; g < G; ++g) fp32[g] += it2[g];
      const float* e_fin = (inner_passes & 1) ? op->e_b : op->e_a;
      hipLaunchKernelGGL(k_graph_update, dim3(grid_for(n)), dim3(kBlock), 0, st, X, zX, Y, zY,
                         e_fin, op->invden, op->graph_of, op->gdone, n);
      PSI_HIP_CHECK(hipGetLastError());
    }
  }
  if (psi_out) {
    PassArgs a = base_args(op);
    a.count_iter = 0;
    a.respect_done = 0;
    a.gskip = nullptr;  // ψ needs every graph's sums
    a.x = z_fin;
    a.s_new = psi_out;
    s = S > 1 ? launch_pass_seg(op, kFinal64G, a, st) : launch_pass(op, kFinal64G, a, st);
    if (s != PSI_OK) return s;
  }
  std::vector<int> it(G), stv(G);
  std::vector<double> gap(G);
  PSI_HIP_CHECK(hipMemcpyAsync(it.data(), op->giter, 4 * size_t(G), hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipMemcpyAsync(stv.data(), op->gstatus, 4 * size_t(G), hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipMemcpyAsync(gap.data(), op->ggap, 8 * size_t(G), hipMemcpyDeviceToHost, st));
  std::vector<int> dn(G);
  PSI_HIP_CHECK(hipMemcpyAsync(dn.data(), op->gdone, 4 * size_t(G), hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipEventRecord(ev1, st));
  PSI_HIP_CHECK(hipEventSynchronize(ev1));
  float ms = 0.f;
  PSI_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
  if (ms_out) *ms_out = ms;
  s = check_waits(op, st);
  if (s != PSI_OK) return s;
  int worst = PSI_OK;
  for (int g = 0; g < G; ++g) {
    const int stg = dn[g] ? stv[g] : PSI_ENOTCONV;
    if (stg != PSI_OK && worst == PSI_OK) worst = stg;
    if (infos) {
      psi_info& inf = infos[g];
      inf = psi_info{};
      inf.status = stg;
      inf.iterations = it[g];
      inf.fp32_passes = fp32[g];
      inf.refinements = refine[g];
      inf.spmv_passes = it[g] + fp32[g] + 1;
      inf.final_gap = gap[g];
      inf.final_l1_step = gap[g];
      inf.col_segments = S;
      inf.seg_form = form;
      inf.tile_items = tile;
      inf.device_ms = ms;
    }
  }
  if (worst != PSI_OK) set_error("a graph did not converge (see its info)");
  return static_cast<psi_status>(worst);
}

psi_status solve_graphs(psi_operator* op, const psi_params* prm, double* psi_out, psi_info* infos,
                        hipStream_t st) {
  PSI_REQUIRE(psi_out, "psi_out must not be NULL");
  return graph_solve(op, prm, psi_out, infos, st, nullptr);
}

psi_status solve_origins(psi_operator* op, const psi_params* prm, int K, const int32_t* origins,
                         double* p_out, double* psi_out, psi_info* infos, void* ws,
                         size_t ws_bytes, hipStream_t st) {
  PSI_REQUIRE(prm && psi_out && ws && origins, "params, origins, psi_out and workspace must not be NULL");
  PSI_REQUIRE(K >= 1, "n_origins must be >= 1");
  PSI_REQUIRE(prm->tol > 0.0 && std::isfinite(prm->tol), "tol must be finite and > 0");
  PSI_REQUIRE(prm->max_iter > 0, "max_iter must be > 0");
  PSI_REQUIRE(prm->tol_mode == PSI_TOL_ABS_L1, "origin batches use PSI_TOL_ABS_L1 (p-tolerance)");
  PSI_REQUIRE(prm->precision == PSI_PREC_FP64, "origin batches run in PSI_PREC_FP64");
  PSI_REQUIRE(op->n_graphs == 1, "origin batches need a single-graph operator");
  const int64_t n = op->n, m = op->m;
  for (int k = 0; k < K; ++k)
    PSI_REQUIRE(origins[k] >= 0 && origins[k] < n, "every origin must be a user id in [0, n)");
  size_t need = batch_layout(n, m, nullptr, nullptr, false);
  if (ws_bytes < need) {
    set_error("workspace smaller than psi_batched_workspace_size reported");
    return PSI_ENOSPACE;
  }
  BatchWs w{};
  batch_layout(n, m, &w, static_cast<char*>(ws), false);
  BSched sc{};
  psi_status s = batch_schedule(op->fm_row_ptr, n, m, w, kWaveItems, kChunkEdges, st,
                                &sc);  // CSR(A): rows = followers
  if (s != PSI_OK) return s;
  struct Pinned {
    BatchCtrl* p = nullptr;
    ~Pinned() {
      if (p) (void)hipHostFree(p);
    }
  } pinned;
  PSI_HIP_CHECK(hipHostMalloc(reinterpret_cast<void**>(&pinned.p), sizeof(BatchCtrl),
                              hipHostMallocDefault));
  BatchCtrl* h = pinned.p;
  const int grid = std::min(rows_grid(), static_cast<int>(sc.n_wtiles));
  const int cgrid = static_cast<int>(std::min<int64_t>(kMaxGrid, (n + 3) / 4));
  EventPair evp;
  PSI_HIP_CHECK(hipEventCreate(&evp.a));
  PSI_HIP_CHECK(hipEventCreate(&evp.b));
  hipEvent_t ev0 = evp.a, ev1 = evp.b;
  PSI_HIP_CHECK(hipEventRecord(ev0, st));
  int worst = PSI_OK;
  for (int k0 = 0; k0 < K; k0 += kMaxK) {
    const int Kc = std::min(kMaxK, K - k0);
    const int64_t nk = n * Kc;
    PSI_HIP_CHECK(hipMemcpyAsync(w.origin, origins + k0, 4 * size_t(Kc), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_bctrl_init, dim3(1), dim3(1), 0, st, w.ctrl, prm->tol, prm->max_iter);
    hipLaunchKernelGGL(k_bzero, dim3(grid_for(nk)), dim3(kBlock), 0, st, w.s_a, w.z_a, nk);
    BArgs base{};
    base.row_ptr = op->fm_row_ptr;
    base.col = op->fm_col;
    base.n_rows = static_cast<int>(n);
    base.Kc = Kc;
    base.row_tiles = w.row_tiles;
    base.n_wtiles = static_cast<int>(sc.n_wtiles);
    base.hub_rows = w.hub_rows;
    base.hub_chunk0 = w.hub_chunk0;
    base.n_hubs = static_cast<int>(sc.n_hubs);
    base.chunk_row = w.chunk_row;
    base.chunk_e0 = w.chunk_e0;
    base.n_chunks = static_cast<int>(sc.n_chunks);
    base.chunk_edges = kChunkEdges;
    base.mu = op->mu;
    base.invden = op->invden;
    base.lam = op->lam;
    base.chunk_part = w.chunk_part;
    base.gap_blk = w.gap_blk;
    base.gap_hub = w.gap_hub;
    base.gap_lvl = w.gap_lvl;
    base.ctrl = w.ctrl;
    base.origin = w.origin;
    // pass i reads buffer set i % 2 and writes the other; pass 0 turns P = 0 into P = B
    // (Algorithm 1's start) and is not an iteration, so it reports no gap
    auto pass = [&](int i, bool gap) -> psi_status {
      BArgs a = base;
      const bool even = (i & 1) == 0;
      a.z = even ? w.z_a : w.z_b;
      a.s_old = even ? w.s_a : w.s_b;
      a.s_new = even ? w.s_b : w.s_a;
      a.z_new = even ? w.z_b : w.z_a;
      launch_spmm<kOrig>(a, grid, st);
      if (gap) launch_batch_gap(a, grid, hub_blocks(a), st);
      PSI_HIP_CHECK(hipGetLastError());
      return PSI_OK;
    };
    s = pass(0, false);
    if (s != PSI_OK) return s;
    int enq = 0, chunk = prm->check_every > 0 ? prm->check_every : 8;
    while (true) {
      const int cnt = std::min(chunk, prm->max_iter - enq);
      for (int i = 0; i < cnt; ++i) {
        s = pass(1 + enq + i, true);
        if (s != PSI_OK) return s;
      }
      enq += cnt;
      PSI_HIP_CHECK(hipMemcpyAsync(h, w.ctrl, sizeof(BatchCtrl), hipMemcpyDeviceToHost, st));
      PSI_HIP_CHECK(hipStreamSynchronize(st));
      if (h->c.done || enq >= prm->max_iter) break;
      if (prm->check_every == 0) chunk = std::min(2 * chunk, 64);
    }
    // passes after the last origin converged exit at once: the result is the
    // output of pass h->c.iter
    const double* P = (h->c.iter & 1) == 0 ? w.s_b : w.s_a;
    hipLaunchKernelGGL(k_origin_colsum, dim3(cgrid), dim3(kBlock), 0, st, P, op->c, n, Kc, K, k0,
                       p_out, w.gap_blk);
    hipLaunchKernelGGL(k_origin_psi, dim3(1), dim3(64), 0, st, w.gap_blk, cgrid, Kc, w.origin,
                       op->d, 1.0 / static_cast<double>(n), psi_out + k0);
    PSI_HIP_CHECK(hipGetLastError());
    for (int k = 0; k < Kc; ++k) {
      int stk = h->kdone[k] ? h->kstatus[k] : PSI_ENOTCONV;
      if (stk != PSI_OK && worst == PSI_OK) worst = stk;
      if (infos) {
        psi_info& inf = infos[k0 + k];
        inf = psi_info{};
        inf.status = stk;
        inf.iterations = h->kiter[k];
        inf.spmv_passes = h->kiter[k] + 1;
        inf.final_gap = h->kgap[k];
        inf.final_l1_step = h->kgap[k];
        inf.col_segments = 1;
        inf.tile_items = kWaveItems;
        inf.batch_tile = kMaxK;
        inf.hub_chunk = kChunkEdges;
      }
    }
  }
  PSI_HIP_CHECK(hipEventRecord(ev1, st));
  PSI_HIP_CHECK(hipEventSynchronize(ev1));
  float ms = 0.f;
  PSI_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
  if (infos)
    for (int k = 0; k < K; ++k) infos[k].device_ms = ms;
  if (worst != PSI_OK) set_error("an origin did not converge (see its info)");
  return static_cast<psi_status>(worst);
}

// Scenario batches: the schedule whose pass over all K scenarios is fastest.
// A candidate is timed on the operator's own rates in every scenario, with a
// control block that never converges: the FP64 step pass (PSI_PREC_FP64) or
// the FP32 correction pass that dominates a mixed solve (PSI_PREC_MIXED),
// each with its gap kernels, times ceil(K / Kc) tiles.  The search is by
// coordinates: scenarios per tile (8, 16, 32, 64 and K, up to 64), then
// items per wave tile (128 to 1024), then edges per hub chunk (512 to 4096).
psi_status autotune_batched(psi_operator* op, int precision, int K, void* ws, size_t ws_bytes,
                            int reps, int* batch_tile, int* batch_items, int* hub_chunk,
                            double* best_ms, hipStream_t st) {
  PSI_REQUIRE(op->n_graphs == 1, "scenario batches need a single-graph operator");
  PSI_REQUIRE(precision == PSI_PREC_FP64 || precision == PSI_PREC_MIXED,
              "batched solves run in PSI_PREC_FP64 or PSI_PREC_MIXED");
  PSI_REQUIRE(K >= 1, "n_scenarios must be >= 1");
  PSI_REQUIRE(ws, "workspace must not be NULL");
  PSI_REQUIRE(reps >= 0, "reps must be >= 0");
  const bool mixed = precision == PSI_PREC_MIXED;
  if (ws_bytes < batch_layout(op->n, op->m, nullptr, nullptr, mixed)) {
    set_error("batched workspace smaller than psi_batched_workspace_size reported");
    return PSI_ENOSPACE;
  }
  BatchWs w{};
  batch_layout(op->n, op->m, &w, static_cast<char*>(ws), mixed);
  const int64_t n = op->n, m = op->m;
  EventPair tm;
  PSI_HIP_CHECK(hipEventCreate(&tm.a));
  PSI_HIP_CHECK(hipEventCreate(&tm.b));
  // mean ms of one pass of a tile of Kc scenarios in the schedule (items, chunk)
  auto time_tile = [&](int Kc, int items, int chunk, double* ms) -> psi_status {
    BSched sc{};
    psi_status s = batch_schedule(op->row_ptr, n, m, w, items, chunk, st, &sc);
    if (s != PSI_OK) return s;
    const int64_t nk = n * Kc;
    hipLaunchKernelGGL(k_bprep_rep, dim3(grid_for(nk)), dim3(kBlock), 0, st, op->lam, op->mu, n,
                       Kc, w.lam, w.mu);
    hipLaunchKernelGGL(k_bprep_den, dim3(grid_for(n * 64)), dim3(kBlock), 0, st, op->fm_row_ptr,
                       op->fm_col, w.lam, w.mu, n, Kc, w.invden, w.c, w.d);
    hipLaunchKernelGGL(k_binit, dim3(grid_for(nk)), dim3(kBlock), 0, st, w.c, w.invden, nk,
                       w.s_a, w.z_a);
    BArgs a = scenario_args(op, w, sc, Kc, chunk);
    if (mixed) {
      hipLaunchKernelGGL(k_bprep32, dim3(grid_for(nk)), dim3(kBlock), 0, st, w.mu, w.invden, nk,
                         w.mu32, w.invden32);
      hipLaunchKernelGGL(k_bprep_inner, dim3(grid_for(nk)), dim3(kBlock), 0, st, w.s_a, w.z_a,
                         w.invden32, nk, w.r32, w.e_a, w.ze_a);
      hipLaunchKernelGGL(k_bctrl_init, dim3(1), dim3(1), 0, st, w.ctrl2, -1.0, INT32_MAX);
      a.ctrl = w.ctrl2;
      a.z32 = w.ze_a;
      a.e_old = w.e_a;
      a.e_new = w.e_b;
      a.ze_new = w.ze_b;
    } else {
      hipLaunchKernelGGL(k_bctrl_init, dim3(1), dim3(1), 0, st, w.ctrl, -1.0, INT32_MAX);
      a.z = w.z_a;
      a.s_old = w.s_a;
      a.s_new = w.s_b;
      a.z_new = w.z_b;
    }
    const int grid = std::min(rows_grid(), static_cast<int>(sc.n_wtiles));
    auto pass = [&]() {
      if (mixed) launch_spmm<kScen32>(a, grid, st);
      else launch_spmm<kScen>(a, grid, st);
      launch_batch_gap(a, grid, hub_blocks(a), st);
    };
    pass();  // warm-up
    int r = reps;
    if (r == 0) {  // about 20 ms of passes, at least 3
      PSI_HIP_CHECK(hipEventRecord(tm.a, st));
      pass();
      PSI_HIP_CHECK(hipEventRecord(tm.b, st));
      PSI_HIP_CHECK(hipEventSynchronize(tm.b));
      float one = 0.f;
      PSI_HIP_CHECK(hipEventElapsedTime(&one, tm.a, tm.b));
      r = static_cast<int>(std::min(50.0, std::max(3.0, 20.0 / std::max<double>(one, 1e-3))));
    }
    PSI_HIP_CHECK(hipEventRecord(tm.a, st));
    for (int i = 0; i < r; ++i) pass();
    PSI_HIP_CHECK(hipEventRecord(tm.b, st));
    PSI_HIP_CHECK(hipEventSynchronize(tm.b));
    PSI_HIP_CHECK(hipGetLastError());
    float tot = 0.f;
    PSI_HIP_CHECK(hipEventElapsedTime(&tot, tm.a, tm.b));
    *ms = tot / r;
    return PSI_OK;
  };
  int bt = std::min(K, kMaxK), bi = kWaveItems, bc = kChunkEdges;
  double best = 0.0;
  auto consider = [&](int Kc, int items, int chunk) -> psi_status {
    double ms = 0.0;
    psi_status s = time_tile(Kc, items, chunk, &ms);
    if (s != PSI_OK) return s;
    const double total = ms * static_cast<double>((K + Kc - 1) / Kc);
    if (best == 0.0 || total < best) {
      best = total;
      bt = Kc;
      bi = items;
      bc = chunk;
    }
    return PSI_OK;
  };
  std::vector<int> tiles;
  for (int Kc : {8, 16, 32, 64})
    if (Kc < std::min(K, kMaxK)) tiles.push_back(Kc);
  tiles.push_back(std::min(K, kMaxK));
  for (int Kc : tiles) {
    psi_status s = consider(Kc, kWaveItems, kChunkEdges);
    if (s != PSI_OK) return s;
  }
  const int Kb = bt;
  for (int items : {128, 512, 1024}) {
    psi_status s = consider(Kb, items, kChunkEdges);
    if (s != PSI_OK) return s;
  }
  const int Ib = bi;
  for (int chunk : {512, 2048, 4096}) {
    psi_status s = consider(Kb, Ib, chunk);
    if (s != PSI_OK) return s;
  }
  op->tuned_batch_tile[precision] = bt;
  op->tuned_batch_items[precision] = bi;
  op->tuned_batch_chunk[precision] = bc;
  if (batch_tile) *batch_tile = bt;
  if (batch_items) *batch_items = bi;
  if (hub_chunk) *hub_chunk = bc;
  if (best_ms) *best_ms = best;
  return PSI_OK;
}

// Graph batches: the schedule (tile items, column segments, partial-pass
// form) whose whole batch solve to `tol` is fastest (without the final ψ
// pass).  Whole solves, not single passes, are timed: graphs freeze as they
// converge, and only the tiled forms skip the gathers of frozen graphs, so the
// fastest pass over a fully live batch need not give the fastest solve.
psi_status autotune_graphs(psi_operator* op, int precision, double tol, int reps,
                           int* tile_items, int* col_segments, int* seg_form, double* best_ms,
                           hipStream_t st) {
  PSI_REQUIRE(op->n_graphs > 1, "graph mode needs a multi-graph operator");
  PSI_REQUIRE(precision == PSI_PREC_FP64 || precision == PSI_PREC_MIXED,
              "graph batches run in PSI_PREC_FP64 or PSI_PREC_MIXED");
  PSI_REQUIRE(tol > 0.0 && std::isfinite(tol), "tol must be finite and > 0");
  PSI_REQUIRE(reps >= 0, "reps must be >= 0");
  const bool mixed = precision == PSI_PREC_MIXED;
  // the candidates run with these explicit schedules; what a failing
  // candidate leaves tuned is cleared first
  op->tuned_graph_S[precision] = 0;
  auto time_one = [&](int tile, int S, int form, double* ms) -> psi_status {
    psi_params p{};
    p.tol = tol;
    p.tol_mode = PSI_TOL_ABS_L1;
    p.max_iter = 100000;
    p.precision = precision;
    p.tile_items = tile;
    p.col_segments = S;
    p.seg_form = form == 0 ? 0 : form;
    if (S == 1) p.seg_form = 0;
    float one = 0.f;
    psi_status s = graph_solve(op, &p, nullptr, nullptr, st, &one);  // warm-up
    if (s != PSI_OK && s != PSI_ENOTCONV) return s;
    const int r = std::max(1, reps);
    double tot = 0.0;
    for (int i = 0; i < r; ++i) {
      s = graph_solve(op, &p, nullptr, nullptr, st, &one);
      if (s != PSI_OK && s != PSI_ENOTCONV) return s;
      tot += one;
    }
    *ms = tot / r;
    return PSI_OK;
  };
  static const int kTiles[] = {1024, 2048, 3072, 4096};
  double best = 0.0;
  int bt = 0, bS = 0, bf = 0, tile_s1 = kDefaultTileItems;
  double best_s1 = 0.0;
  for (int S : {1, 2, 4, 8}) {
    if (mixed && S == 8) break;  // the FP32 pass takes at most four segments
    for (int tile : kTiles) {
      double ms = 0.0;
      psi_status s = time_one(tile, S, S > 1 ? kSegTiles : 0, &ms);
      if (s != PSI_OK) return s;
      if (S == 1 && (best_s1 == 0.0 || ms < best_s1)) {
        best_s1 = ms;
        tile_s1 = tile;
      }
      if (best == 0.0 || ms < best) {
        best = ms;
        bt = tile;
        bS = S;
        bf = S > 1 ? kSegTiles : 0;
      }
    }
    if (S > 1) {
      double ms = 0.0;
      psi_status s = time_one(tile_s1, S, kSegSlices, &ms);
      if (s != PSI_OK) return s;
      if (ms < best) {
        best = ms;
        bt = tile_s1;
        bS = S;
        bf = kSegSlices;
      }
    }
  }
  op->tuned_graph_tile[precision] = bt;
  op->tuned_graph_S[precision] = bS;
  op->tuned_graph_form[precision] = bf;
  if (tile_items) *tile_items = bt;
  if (col_segments) *col_segments = bS;
  if (seg_form) *seg_form = bf;
  if (best_ms) *best_ms = best;
  return PSI_OK;
}

}  // namespace psi
