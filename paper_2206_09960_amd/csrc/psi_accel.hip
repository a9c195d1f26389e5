// Anderson-accelerated Power-ψ: the fixed point s = Aᵀs + c of eq. (power_psi)
// found with fewer operator passes.
//
// Each iteration is one Power-ψ pass g_k = Aᵀx_k + c (the same kernels as
// Algorithm 2) followed by Anderson mixing (Anderson, J. ACM 1965; Walker &
// Ni, SIAM J. Numer. Anal. 2011) over the last m residuals f = g − x:
//
//   ΔF = [f_{k−j+1} − f_{k−j}], ΔG = [g_{k−j+1} − g_{k−j}] (j = 1..m_k),
//   γ = argmin ‖f_k − ΔF γ‖₂,   x_{k+1} = g_k − ΔG γ.
//
// For a linear map this is a windowed Krylov method, so the passes needed for
// a given accuracy fall well below the power iteration's.  The stopping test
// is the pass's own gap ‖g_k − x_k‖₁ ≤ ε (the s-tolerance of eq. condition,
// in any PSI_TOL_* unit), and the result is s = g_k: one Power-ψ step from
// x_k of size at most ε, exactly the criterion Algorithm 2 applies to its
// last step.  ψ = (Bᵀs + d)/N follows as in Algorithm 2.
//
// Device work per iteration: the pass, which leaves its gap as per-workgroup
// pairs; k_aa_diff (its workgroup 0 first decides the pass's gap; then f,
// ΔF, ΔG into a ring of m columns, and the 2m dot products ⟨ΔF_j, ΔF_new⟩,
// ⟨ΔF_j, f⟩ as per-workgroup partials); k_aa_solve (one workgroup: the
// partials in fixed order, the Gram matrix updated by one row/column, a
// Cholesky solve with a small relative shift; the window is cleared if the
// factorisation fails or the gap grows tenfold); k_aa_mix (x_{k+1},
// z = x/den).  Every reduction has a fixed order, so solves are bitwise
// repeatable.
//
// In mixed precision the same mixing accelerates each FP32 correction solve
// e = Aᵀe + r between the FP64 residual passes of the refinement (the
// iteration of psi_solve's PSI_PREC_MIXED): the window's columns, f and g are
// FP32, every dot product and the mixing sum are FP64, and the window starts
// empty for every correction.
#include <algorithm>
#include <cmath>
#include <limits>

#include <mutex>
#include <string>

#include "psi_internal.h"

namespace psi {

namespace {

constexpr int kMaxDepth = 8;
constexpr int kAaGrid = 2048;       // most workgroups of k_aa_diff (one partial row each)
constexpr int kAaSolveBlock = 1024; // threads of k_aa_solve

inline unsigned grid_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }
inline size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

struct AaState {
  int valid;      // f_prev, g_prev hold the previous iteration
  int count;      // columns in the window
  int head;       // ring slot that the next column takes
  int restarts;
  double best;    // smallest gap seen
  double G[kMaxDepth][kMaxDepth];  // Gram matrix of ΔF, by ring slot
  double gamma[kMaxDepth];          // mixing coefficients, by ring slot
};

struct AaWs {
  double* dF;      // [m × N]
  double* dG;      // [m × N]
  double* f_prev;  // [N]
  double* g_prev;  // [N]
  double* part;    // [kAaGrid × 2m]
  AaState* st;
};

// The window's vectors in the iterate's type (FP32 ones use the first half of
// each FP64 array).
template <class T>
struct AaVecs {
  T* dF;
  T* dG;
  T* f_prev;
  T* g_prev;
};

template <class T>
AaVecs<T> aa_vecs(const AaWs& w) {
  return AaVecs<T>{reinterpret_cast<T*>(w.dF), reinterpret_cast<T*>(w.dG),
                   reinterpret_cast<T*>(w.f_prev), reinterpret_cast<T*>(w.g_prev)};
}

size_t aa_layout(int64_t n, int m, AaWs* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(std::max<size_t>(bytes, 1));
    return p;
  };
  AaWs t{};
  t.dF = (double*)take(8 * size_t(m) * size_t(n));
  t.dG = (double*)take(8 * size_t(m) * size_t(n));
  t.f_prev = (double*)take(8 * size_t(n));
  t.g_prev = (double*)take(8 * size_t(n));
  t.part = (double*)take(8 * size_t(kAaGrid) * 2 * kMaxDepth);
  t.st = (AaState*)take(sizeof(AaState));
  if (w) *w = t;
  return off;
}

__global__ void k_aa_init(AaState* s) {
  s->valid = 0;
  s->count = 0;
  s->head = 0;
  s->restarts = 0;
  s->best = INFINITY;
  for (int i = 0; i < kMaxDepth; ++i) {
    s->gamma[i] = 0.0;
    for (int j = 0; j < kMaxDepth; ++j) s->G[i][j] = 0.0;
  }
}

// f = g − x; the new ΔF, ΔG column at ring slot `head`; f_prev, g_prev ← f, g;
// partial dot products (FP64) of every window column (the new one included)
// with the new ΔF column and with f.
template <class T>
__global__ __launch_bounds__(kBlock) void k_aa_diff(const T* g, const T* x, int64_t n, int m,
                                                    AaVecs<T> v, AaWs w, Ctrl* ctrl,
                                                    double* pairs, double* hist) {
  __shared__ double red[2 * (kBlock / 64)];
  __shared__ int s_done;
  // the pass's gap: decided here, before k_aa_solve reads it
  if (blockIdx.x == 0) take_deferred(ctrl, pairs, hist, 1, -1, red);
  // one reading per workgroup.  A decision by workgroup 0 just now may reach
  // some workgroups and not others, which is harmless: once done, nothing
  // later in the solve reads what this kernel writes.
  if (threadIdx.x == 0) s_done = ctrl->done;
  __syncthreads();
  if (s_done) return;
  const int valid = w.st->valid, slot = w.st->head;  // uniform
  const int cnt = valid ? std::min(w.st->count + 1, m) : 0;
  double vv[kMaxDepth], vb[kMaxDepth];
#pragma unroll
  for (int j = 0; j < kMaxDepth; ++j) vv[j] = vb[j] = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const T gi = g[i], fi = gi - x[i];
    if (valid) {
      const T df = fi - v.f_prev[i];
      v.dF[int64_t(slot) * n + i] = df;
      v.dG[int64_t(slot) * n + i] = gi - v.g_prev[i];
#pragma unroll
      for (int q = 0; q < kMaxDepth; ++q) {
        if (q < cnt) {  // window column q: q steps back from the new one
          const int sj = (slot - q + m) % m;
          const double dj = static_cast<double>(q == 0 ? df : v.dF[int64_t(sj) * n + i]);
          vv[q] += dj * static_cast<double>(df);
          vb[q] += dj * static_cast<double>(fi);
        }
      }
    }
    v.f_prev[i] = fi;
    v.g_prev[i] = gi;
  }
  if (!valid) return;  // uniform: no dot products on the first iteration
  // all 2m sums at once: wave shuffles, one LDS round, waves added in order
  __shared__ double wsum[kBlock / 64][2 * kMaxDepth];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kMaxDepth; ++q) {
    if (q >= cnt) break;  // uniform
    double a = vv[q], b = vb[q];
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b += __shfl_down(b, off, 64);
    }
    if (lane == 0) {
      wsum[wave][q] = a;
      wsum[wave][kMaxDepth + q] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * kMaxDepth && (threadIdx.x % kMaxDepth) < cnt) {
    const int q = threadIdx.x;
    w.part[int64_t(blockIdx.x) * 2 * kMaxDepth + q] =
        (wsum[0][q] + wsum[1][q]) + (wsum[2][q] + wsum[3][q]);
  }
}

// One workgroup: reduce the partials (64 interleaved slices with every load
// in flight at once, then the slices in order), update the Gram matrix, and
// solve (G + δI) γ = b over the window by Cholesky.
__global__ __launch_bounds__(kAaSolveBlock) void k_aa_solve(AaWs w, int m, int n_blk,
                                                           const Ctrl* ctrl) {
  constexpr int kCols = 2 * kMaxDepth;
  constexpr int kSlices = kAaSolveBlock / kCols;
  constexpr int kPer = kAaGrid / kSlices;  // partial rows per slice at most
  __shared__ double v[kCols];
  __shared__ double slice[kSlices][kCols];
  if (ctrl->done) return;
  AaState* st = w.st;
  // every thread reads the state before thread 0 changes it
  const int valid = st->valid;
  const int cnt = std::min(st->count + 1, m);
  __syncthreads();
  if (!valid) {  // uniform
    if (threadIdx.x == 0) {
      st->valid = 1;
      st->count = 0;
      st->best = ctrl->gap;
    }
    return;
  }
  {
    const int q = threadIdx.x % kCols, sl = threadIdx.x / kCols;
    double part[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int b = sl + k * kSlices;
      part[k] = (q % kMaxDepth) < cnt && b < n_blk ? w.part[int64_t(b) * kCols + q] : 0.0;
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) s += part[k];
    slice[sl][q] = s;
    __syncthreads();
    if (threadIdx.x < kCols) {
      double t = 0.0;
      for (int k = 0; k < kSlices; ++k) t += slice[k][threadIdx.x];
      v[threadIdx.x] = t;
    }
    __syncthreads();
  }
  // the window's state in LDS; thread 0 then works there (no scratch, no
  // dependent global loads)
  __shared__ double Gs[kMaxDepth][kMaxDepth];
  __shared__ double Ls[kMaxDepth][kMaxDepth];
  __shared__ double ys[kMaxDepth];
  if (threadIdx.x < kMaxDepth * kMaxDepth)
    Gs[threadIdx.x / kMaxDepth][threadIdx.x % kMaxDepth] =
        st->G[threadIdx.x / kMaxDepth][threadIdx.x % kMaxDepth];
  __syncthreads();
  if (threadIdx.x != 0) return;
  const int slot = st->head;
  // column / row of the new slot; window column q sits at slot (slot − q) mod m
  for (int k = 0; k < cnt; ++k) {
    const int sj = (slot - k + m) % m;
    Gs[slot][sj] = v[k];
    Gs[sj][slot] = v[k];
  }
  st->head = (slot + 1) % m;
  st->count = cnt;
  const double gap = ctrl->gap;
  bool ok = gap <= 10.0 * st->best;
  if (gap < st->best) st->best = gap;
  // Cholesky of the window's Gram matrix (order: newest first) with a shift
  double tr = 0.0;
  for (int a = 0; a < cnt; ++a) {
    const int sa = (slot - a + m) % m;
    tr += Gs[sa][sa];
  }
  const double shift = 1e-13 * tr / cnt;
  for (int a = 0; a < cnt && ok; ++a) {
    const int sa = (slot - a + m) % m;
    for (int b = 0; b <= a; ++b) {
      const int sb = (slot - b + m) % m;
      double sum = Gs[sa][sb] + (a == b ? shift : 0.0);
      for (int k = 0; k < b; ++k) sum -= Ls[a][k] * Ls[b][k];
      if (a == b) {
        if (!(sum > 0.0) || !isfinite(sum)) {
          ok = false;
          break;
        }
        Ls[a][a] = sqrt(sum);
      } else {
        Ls[a][b] = sum / Ls[b][b];
      }
    }
  }
  if (ok) {
    for (int a = 0; a < cnt; ++a) {  // L y = b
      double sum = v[kMaxDepth + a];
      for (int k = 0; k < a; ++k) sum -= Ls[a][k] * ys[k];
      ys[a] = sum / Ls[a][a];
    }
    for (int a = cnt - 1; a >= 0; --a) {  // Lᵀ γ = y
      double sum = ys[a];
      for (int k = a + 1; k < cnt; ++k) sum -= Ls[k][a] * ys[k];
      ys[a] = sum / Ls[a][a];
    }
  } else {  // clear the window: the next step is a plain Power-ψ step
    st->count = 0;
    st->restarts += 1;
  }
  // window column a sits at ring slot (slot − a) mod m; slots outside it get γ = 0
  for (int sj = 0; sj < kMaxDepth; ++sj) st->gamma[sj] = 0.0;
  if (ok)
    for (int a = 0; a < cnt; ++a) st->gamma[(slot - a + m) % m] = ys[a];
  for (int i = 0; i < kMaxDepth; ++i)
    for (int j = 0; j < kMaxDepth; ++j) st->G[i][j] = Gs[i][j];
}

// x_{k+1} = g_k − ΔG γ (summed in FP64) and its gathered form z = x/den.
template <class T>
__global__ __launch_bounds__(kBlock) void k_aa_mix(const T* g, const T* invden, int64_t n, int m,
                                                   AaVecs<T> vw, AaWs w, T* x, T* z,
                                                   const Ctrl* ctrl) {
  if (ctrl->done) return;
  const int cnt = w.st->count;
  double gam[kMaxDepth];
#pragma unroll
  for (int j = 0; j < kMaxDepth; ++j) gam[j] = j < m ? w.st->gamma[j] : 0.0;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  double v = static_cast<double>(g[i]);
  if (cnt > 0) {
    // slots outside the window have γ = 0 and may never have been written
#pragma unroll
    for (int j = 0; j < kMaxDepth; ++j)
      if (j < m && gam[j] != 0.0) v -= gam[j] * static_cast<double>(vw.dG[int64_t(j) * n + i]);
  }
  const T xv = static_cast<T>(v);
  x[i] = xv;
  z[i] = invden[i] * xv;
}

__global__ void k_aa_start(const double* s0, const double* c, const double* invden, int64_t n,
                           double* s, double* z) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = s0 ? s0[i] : c[i];
  s[i] = v;
  z[i] = invden[i] * v;
}

__global__ void k_aa_ctrl(Ctrl* c, double tol, int tol_mode, int max_iter, double bnorm) {
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

}  // namespace

// ---------------------------------------------------------------- no-allocation entry
// Scratch of psi_solve_anderson_noalloc: a file-scope device array, so that a
// caller that cannot allocate device memory can still run the Anderson
// solve.  Each device the library runs on holds its own copy until the
// process ends; its address on a device comes from hipGetSymbolAddress with
// that device current (the array's name in host code is only a stand-in).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};
}  // namespace

// Device address of the scratch array on device `dev` (current), looked up
// once per device.
psi_status noalloc_scratch(int dev, void** ptr, size_t* bytes) {
  PSI_REQUIRE(dev >= 0 && dev < 64, "device index out of range for the no-allocation scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    PSI_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  *bytes = kNoAllocScratchBytes;
  return PSI_OK;
}

psi_status solve_anderson_noalloc(psi_operator* op, const psi_params* prm, int depth,
                                  const double* s0, double* psi_out, double* s_out,
                                  psi_info* info, hipStream_t st) {
  PSI_REQUIRE(depth >= 1 && depth <= kMaxDepth, "depth must be in [1, 8]");
  const size_t need = aa_layout(op->n, depth, nullptr, nullptr);
  if (need > kNoAllocScratchBytes) {
    set_error("psi_solve_anderson_noalloc: " + std::to_string(op->n) + " users at depth " +
              std::to_string(depth) + " need " + std::to_string(need) +
              " bytes of scratch, more than its fixed " +
              std::to_string(kNoAllocScratchBytes) + " (use psi_solve_anderson)");
    return PSI_ENOSPACE;
  }
  void* ws = nullptr;
  size_t bytes = 0;
  psi_status s = noalloc_scratch(op->device, &ws, &bytes);
  if (s != PSI_OK) return s;
  return solve_anderson(op, prm, depth, s0, psi_out, s_out, info, ws, bytes, st);
}

psi_status anderson_workspace_size(const psi_operator* op, int depth, size_t* bytes) {
  PSI_REQUIRE(bytes, "bytes must not be NULL");
  PSI_REQUIRE(depth >= 1 && depth <= kMaxDepth, "depth must be in [1, 8]");
  *bytes = aa_layout(op->n, depth, nullptr, nullptr);
  return PSI_OK;
}

psi_status solve_anderson(psi_operator* op, const psi_params* prm, int depth, const double* s0,
                          double* psi_out, double* s_out, psi_info* info, void* ws,
                          size_t ws_bytes, hipStream_t st) {
  PSI_REQUIRE(prm && psi_out && ws, "params, psi_out and workspace must not be NULL");
  PSI_REQUIRE(depth >= 1 && depth <= kMaxDepth, "depth must be in [1, 8]");
  PSI_REQUIRE(prm->tol > 0.0 && std::isfinite(prm->tol), "tol must be finite and > 0");
  PSI_REQUIRE(prm->max_iter > 0, "max_iter must be > 0");
  PSI_REQUIRE(prm->tol_mode >= PSI_TOL_ABS_L1 && prm->tol_mode <= PSI_TOL_REL_L1,
              "unknown tol_mode");
  PSI_REQUIRE(prm->precision == PSI_PREC_FP64 || prm->precision == PSI_PREC_MIXED,
              "Anderson solves run in PSI_PREC_FP64 or PSI_PREC_MIXED");
  PSI_REQUIRE(op->n_graphs == 1, "Anderson solves need a single-graph operator");
  const size_t need = aa_layout(op->n, depth, nullptr, nullptr);
  if (ws_bytes < need) {
    set_error("workspace smaller than psi_anderson_workspace_size reported");
    return PSI_ENOSPACE;
  }
  AaWs w{};
  aa_layout(op->n, depth, &w, static_cast<char*>(ws));
  const int64_t n = op->n;
  const int prec = prm->precision;
  const bool mixed = prec == PSI_PREC_MIXED;
  const int xbytes = mixed ? 4 : 8;  // gathered element of the passes that dominate
  const int tuned_tile = op->tuned_tile[prec];
  const int tile = prm->tile_items ? prm->tile_items
                 : tuned_tile      ? tuned_tile
                 : (op->sched_items ? op->sched_items : kDefaultTileItems);
  PSI_REQUIRE(tile_items_supported(tile), "unsupported tile_items");
  int S = prm->col_segments ? prm->col_segments : op->tuned_S[prec];
  if (S == 0) {  // the same rule as psi_solve for the gathered vector
    const double xb = static_cast<double>(xbytes) * static_cast<double>(n);
    S = 1;
    if (xb > 3.0e6) {
      S = 2;
      while (S < 8 && xb / S > 2.5e6) S *= 2;
    }
  }
  PSI_REQUIRE(S == 1 || S == 2 || S == 4 || S == 8, "col_segments must be 0, 1, 2, 4 or 8");
  int form = 0;
  psi_status s = resolve_form(op, prm->seg_form, prm->col_segments, prec, S, xbytes, &form);
  if (s != PSI_OK) return s;
  if (form == kSegBands || form == kSegBins) S = 1;
  {
    int wlog = 0, rows = 0;
    if (form == kSegBands) band_params(op, prec, &wlog, &rows);
    if (prm->band_col_log) wlog = prm->band_col_log;
    if (prm->band_rows) rows = prm->band_rows;
    PSI_REQUIRE(form != kSegBands || ((wlog == 17 || wlog == 18) && band_rows_supported(rows)),
                "band_col_log must be 0, 17 or 18 and band_rows 0, 1024 or 2048");
    s = prepare(op, tile, S, form, st, wlog, rows);
    op->band_pace_ticks = form == kSegBands && op->tuned_band_wlog[prec] == wlog &&
                                  op->tuned_band_rows[prec] == rows
                              ? op->tuned_band_pace[prec]
                              : 0ull;
  }
  if (s != PSI_OK) return s;
  auto pass = [&](PassMode mode, const PassArgs& a) { return run_pass(op, S, mode, a, st); };
  EventPair evp;
  PSI_HIP_CHECK(hipEventCreate(&evp.a));
  PSI_HIP_CHECK(hipEventCreate(&evp.b));
  hipEvent_t ev0 = evp.a, ev1 = evp.b;
  PSI_HIP_CHECK(hipEventRecord(ev0, st));
  double* X = op->s_a;
  double* zX = op->z_a;
  double* Gb = op->s_b;
  double* zG = op->z_b;
  hipLaunchKernelGGL(k_aa_start, dim3(grid_for(n)), dim3(kBlock), 0, st, s0, op->c, op->invden,
                     n, X, zX);
  hipLaunchKernelGGL(k_aa_ctrl, dim3(1), dim3(1), 0, st, op->ctrl, prm->tol, prm->tol_mode,
                     prm->max_iter, op->stats.b_norm);
  PSI_HIP_CHECK(hipGetLastError());
  const int dgrid = static_cast<int>(std::min<int64_t>(kAaGrid, (n + kBlock - 1) / kBlock));
  PassArgs base = base_args(op);
  // One accelerated iteration: a pass g = Aᵀx + b from x (FP64 with b = c,
  // or FP32 with b = r), then the window update, the small solve and the mix
  // x ← g − ΔG γ, all under control block `ctrl`.
  auto iteration = [&](bool fp32, Ctrl* ctrl) -> psi_status {
    PassArgs a = base;
    if (fp32) {
      a.x = op->ze_a;
      a.r32 = op->r32;
      a.e_old = op->e_a;
      a.e_new = op->e_b;
      a.ze_new = op->ze_b;
    } else {
      a.x = zX;
      a.s_old = X;
      a.s_new = Gb;
      a.z_new = zG;
    }
    a.count_iter = 1;
    a.respect_done = 1;
    a.ctrl = ctrl;
    a.defer_gap = 1;  // pairs in gap_part, decided by k_aa_diff
    a.gap_prev = op->gap_part + 2 * kMaxGrid;  // nothing is ever pending there
    psi_status r = pass(fp32 ? kStep32 : kStep64, a);
    if (r != PSI_OK) return r;
    if (fp32) {
      const AaVecs<float> v = aa_vecs<float>(w);
      hipLaunchKernelGGL(k_aa_diff<float>, dim3(dgrid), dim3(kBlock), 0, st, op->e_b, op->e_a, n,
                         depth, v, w, ctrl, op->gap_part, op->hist);
      hipLaunchKernelGGL(k_aa_solve, dim3(1), dim3(kAaSolveBlock), 0, st, w, depth, dgrid, ctrl);
      hipLaunchKernelGGL(k_aa_mix<float>, dim3(grid_for(n)), dim3(kBlock), 0, st, op->e_b,
                         op->invden32, n, depth, v, w, op->e_a, op->ze_a, ctrl);
    } else {
      const AaVecs<double> v = aa_vecs<double>(w);
      hipLaunchKernelGGL(k_aa_diff<double>, dim3(dgrid), dim3(kBlock), 0, st, Gb, X, n, depth, v,
                         w, ctrl, op->gap_part, op->hist);
      hipLaunchKernelGGL(k_aa_solve, dim3(1), dim3(kAaSolveBlock), 0, st, w, depth, dgrid, ctrl);
      hipLaunchKernelGGL(k_aa_mix<double>, dim3(grid_for(n)), dim3(kBlock), 0, st, Gb,
                         op->invden, n, depth, v, w, X, zX, ctrl);
    }
    PSI_HIP_CHECK(hipGetLastError());
    return PSI_OK;
  };
  // Runs accelerated iterations from a fresh window until the gap of control
  // block ctrl_idx meets its tolerance (iterations after that exit at once),
  // max_iter is reached or the gap stagnates; blocks of iterations are
  // enqueued between host checks.
  auto accelerate = [&](bool fp32, int ctrl_idx, int max_iter, int* status) -> psi_status {
    Ctrl* ctrl = op->ctrl + ctrl_idx;
    Ctrl* h = op->host_ctrl + ctrl_idx;
    hipLaunchKernelGGL(k_aa_init, dim3(1), dim3(1), 0, st, w.st);
    PSI_HIP_CHECK(hipGetLastError());
    int enq = 0, k = prm->check_every > 0 ? prm->check_every : 4;
    double best = std::numeric_limits<double>::infinity();
    int best_iter = 0;
    *status = PSI_OK;
    while (true) {
      const int cnt = std::min(k, max_iter - enq);
      for (int i = 0; i < cnt; ++i) {
        psi_status r = iteration(fp32, ctrl);
        if (r != PSI_OK) return r;
      }
      enq += cnt;
      PSI_HIP_CHECK(hipMemcpyAsync(h, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
      PSI_HIP_CHECK(hipStreamSynchronize(st));
      if (h->err_flags & kErrSlotTimeout) return check_waits(op, st);
      if (h->done) {
        *status = h->status;
        break;
      }
      if (enq >= max_iter) {
        *status = PSI_ENOTCONV;
        break;
      }
      if (h->gap < best * (1.0 - 1e-3)) {
        best = h->gap;
        best_iter = h->iter;
      } else if (h->iter - best_iter >= 25) {
        *status = PSI_ESTAGNATED;
        break;
      }
      if (prm->check_every == 0) k = std::min(2 * k, 16);
    }
    return PSI_OK;
  };
  psi_info inf{};
  int status = PSI_OK;
  const double* z_fin = zG;
  const double* s_fin = Gb;
  int restarts = 0;
  if (!mixed) {
    s = accelerate(false, 0, prm->max_iter, &status);
    if (s != PSI_OK) return s;
    inf.iterations = op->host_ctrl->iter;
    AaState hs{};
    PSI_HIP_CHECK(hipMemcpyAsync(&hs, w.st, sizeof(AaState), hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    restarts = hs.restarts;
    inf.refinements = restarts;  // window restarts
  } else {
    // FP64 residual passes X → Gb around accelerated FP32 corrections, as
    // psi_solve's PSI_PREC_MIXED; when a refinement stops shrinking the gap
    // fourfold, accelerated FP64 iterations finish from Gb.
    const double eta = prm->inner_tol > 0.0 ? prm->inner_tol : 2e-6;
    double prev_gap = std::numeric_limits<double>::infinity();
    int fp64_passes = 0;
    Ctrl* h = op->host_ctrl;
    while (true) {
      PassArgs a = base;
      a.x = zX;
      a.s_old = X;
      a.s_new = Gb;
      a.z_new = zG;
      a.count_iter = 1;
      a.respect_done = 0;
      a.ctrl = op->ctrl;
      s = pass(kStep64, a);
      if (s != PSI_OK) return s;
      ++fp64_passes;
      s = check_waits(op, st);  // copies both control blocks to the host
      if (s != PSI_OK) return s;
      if (h->done) {
        status = h->status;
        break;
      }
      if (fp64_passes >= prm->max_iter) {
        status = PSI_ENOTCONV;
        break;
      }
      if (!(h->gap < 0.25 * prev_gap)) {
        // refinement no longer gains: accelerated FP64 iterations from Gb
        hipLaunchKernelGGL(k_aa_start, dim3(grid_for(n)), dim3(kBlock), 0, st, Gb, op->c,
                           op->invden, n, X, zX);
        hipLaunchKernelGGL(k_aa_ctrl, dim3(1), dim3(1), 0, st, op->ctrl, prm->tol, prm->tol_mode,
                           prm->max_iter - fp64_passes, op->stats.b_norm);
        PSI_HIP_CHECK(hipGetLastError());
        s = accelerate(false, 0, prm->max_iter - fp64_passes, &status);
        if (s != PSI_OK) return s;
        fp64_passes += h->iter;
        break;
      }
      prev_gap = h->gap;
      s = mixed_inner_begin(op, Gb, X, eta, prm->max_iter, st);
      if (s != PSI_OK) return s;
      int inner_status = PSI_OK;
      s = accelerate(true, 1, prm->max_iter, &inner_status);
      if (s != PSI_OK) return s;
      inf.fp32_passes += op->host_ctrl[1].iter;
      if (inner_status == PSI_ENUMERIC) {
        status = PSI_ENUMERIC;
        break;
      }
      // e = g of the correction's last pass
      s = mixed_update(op, X, op->e_b, zX, st);
      if (s != PSI_OK) return s;
      inf.refinements += 1;
    }
    inf.iterations = fp64_passes;
  }
  // ψ = (Bᵀs + d)/N from s = g of the last FP64 pass (the last line of Algorithm 2)
  {
    PassArgs a = base;
    a.x = z_fin;
    a.s_new = psi_out;
    a.count_iter = 0;
    a.respect_done = 0;
    s = pass(kFinal64, a);
    if (s != PSI_OK) return s;
  }
  if (s_out) PSI_HIP_CHECK(hipMemcpyAsync(s_out, s_fin, 8 * size_t(n), hipMemcpyDeviceToDevice, st));
  PSI_HIP_CHECK(hipEventRecord(ev1, st));
  PSI_HIP_CHECK(hipEventSynchronize(ev1));
  float ms = 0.f;
  PSI_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
  s = check_waits(op, st);
  if (s != PSI_OK) return s;
  const Ctrl* h = op->host_ctrl;
  inf.status = status;
  inf.spmv_passes = inf.iterations + inf.fp32_passes + 1;
  inf.used_s0 = s0 ? 1 : 0;
  inf.col_segments = S;
  inf.tile_items = tile;
  inf.seg_form = form;
  inf.final_gap = h->gap;
  inf.final_l1_step = h->l1;
  inf.b_norm = op->stats.b_norm;
  inf.kappa = op->stats.kappa;
  inf.err_bound_s = inf.kappa < 1.0 ? inf.kappa / (1.0 - inf.kappa) * h->l1
                                    : std::numeric_limits<double>::infinity();
  inf.psi_gap_bound = h->l1 * inf.b_norm / static_cast<double>(n);
  inf.device_ms = ms;
  if (info) *info = inf;
  if (status == PSI_ENOTCONV) set_error("max_iter reached before the gap fell to tol");
  else if (status == PSI_ESTAGNATED) set_error("the gap stopped decreasing above tol");
  else if (status == PSI_ENUMERIC) set_error("NaN or Inf in the iteration");
  return static_cast<psi_status>(status);
}

}  // namespace psi
