// One Power-ψ operator pass: y_i = Σ_{j∈F(i)} x_j over the follower lists of
// CSR(Aᵀ) (the row-vector product sᵀA of eq. power_psi written as a pull),
// fused with the per-user epilogue (the axpy of Algorithm 2, or its last line)
// and the L1 gap of eq. eps_t.
//
// Work split: merge-path tiles (Merrill & Garland, SC'16).  The path merges
// the row ends row_ptr[1..N] with the edge indices 0..M-1; tile b owns path
// items [b·T, (b+1)·T).  Every tile does the same work whatever the degree
// distribution, so the power-law follower counts (hub rows) need no special
// kernel.  Inside a tile:
//   1. coalesced, non-temporal reads of the column indices, one gather of x
//      per edge into LDS (x stays cache-resident);
//   2. each thread consumes T/256 consecutive path items from LDS;
//   3. a segmented scan of the per-thread carries finishes rows that span
//      threads;
//   4. rows that begin and end in the tile get their epilogue at once.
// The grid is persistent and co-resident (cooperative launch): workgroups walk
// the tiles grid-stride.  A row that spans tiles is summed from the tiles'
// partials, in tile order, by the workgroup that owns the tile where the row
// ends; partials travel through coherent slots (see take_slot), so no cache
// flush or floating-point atomic is needed and every pass is bitwise
// repeatable.  The gap is one partial per workgroup, summed in workgroup order
// by the last workgroup to finish, which also decides termination.
#include <algorithm>
#include <cmath>

#include "psi_internal.h"

namespace psi {

namespace {

__device__ inline void st_agent(double* p, double x) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     static_cast<unsigned long long>(__double_as_longlong(x)), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

constexpr unsigned long long kEmpty = kEmptySlot;

// Wait (bounded) until a slot is filled, take its value and empty it again.
// The writer filled it before it announced itself on the counter the caller
// observed, so the wait is short; the bound only guarantees the kernel ends.
__device__ inline double take_slot(double* p, Ctrl* ctrl) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  unsigned long long v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int spin = 0; v == kEmpty && spin < (1 << 22); ++spin) {
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (v == kEmpty) {
    atomicOr(&ctrl->err_flags, kErrSlotTimeout);
    return 0.0;
  }
  __hip_atomic_store(q, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double(static_cast<long long>(v));
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

template <int MODE>
__device__ inline double gather(const PassArgs& a, int j, int e) {
  if constexpr (MODE == kStep32) {
    return static_cast<double>(static_cast<const float*>(a.x)[j]);
  } else if constexpr (MODE == kStep64W) {
    return static_cast<const double*>(a.x)[j] * __builtin_nontemporal_load(a.val64 + e);
  } else {
    return static_cast<const double*>(a.x)[j];
  }
}

// Per-user epilogue; g accumulates |new − old|, s accumulates |new|.
template <int MODE>
__device__ inline void epilogue(const PassArgs& a, int r, double y, double& g, double& s) {
  if constexpr (MODE == kStep64) {
    const double sn = a.c[r] + a.mu[r] * y;
    const double so = a.s_old[r];
    a.s_new[r] = sn;
    a.z_new[r] = a.invden[r] * sn;
    g += fabs(sn - so);
    s += fabs(sn);
  } else if constexpr (MODE == kStep64W) {
    const double sn = a.c[r] + y;
    const double so = a.s_old[r];
    a.s_new[r] = sn;
    g += fabs(sn - so);
    s += fabs(sn);
  } else if constexpr (MODE == kFinal64) {
    a.s_new[r] = (a.lam[r] * y + a.d[r]) * a.inv_n;
  } else {
    const float en = a.r32[r] + a.mu32[r] * static_cast<float>(y);
    const float eo = a.e_old[r];
    a.e_new[r] = en;
    a.ze_new[r] = a.invden32[r] * en;
    g += fabs(static_cast<double>(en) - static_cast<double>(eo));
    s += fabs(static_cast<double>(en));
  }
}

// Finish a row that spans tiles [bs, be]: its partials from tiles bs..be-1
// (published by their blocks) plus this tile's head partial, summed in tile
// order; then its epilogue.  Called by the whole workgroup of the block that
// owns tile be, so the row's gap term lands in a fixed place of the sum.
template <int MODE, int T>
__device__ void finish_row(const PassArgs& a, int r, int be, double head, double* sh, double& g,
                           double& sn) {
  const int bs = static_cast<int>((static_cast<long long>(r) + a.row_ptr[r]) / T);
  double acc = 0.0, dummy = 0.0;
  for (int q = bs + static_cast<int>(threadIdx.x); q < be; q += kBlock)
    acc += take_slot(&a.part_open[q], a.ctrl);
  block_sum2(acc, dummy, sh);
  if (threadIdx.x == 0) epilogue<MODE>(a, r, acc + head, g, sn);
}

// Persistent pass: a co-resident grid walks the tiles grid-stride.  A tile
// publishes the partial of its open last row at once; the row that ends in a
// tile but began earlier is finished one iteration later (its earlier tiles
// were handed out before this one, so their partials are ready by then).
template <int IPT, int MODE>
__global__ __launch_bounds__(kBlock) void k_pass(PassArgs a) {
  constexpr int T = kBlock * IPT;
  __shared__ int s_rowend[T];
  __shared__ double s_val[T];
  __shared__ double s_rowval[T];
  __shared__ int s_crow[kBlock];
  __shared__ double s_cval[kBlock];
  __shared__ double s_red[8];
  __shared__ int s_last;

  if (a.respect_done && a.ctrl->done) return;
  const int tid = threadIdx.x;
  const long long total = static_cast<long long>(a.n_rows) + a.n_nnz;
  double g = 0.0, sn = 0.0;
  int pend_row = -1, pend_tile = 0;  // uniform across the workgroup
  double pend_head = 0.0;

  for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int r0 = a.tile_row[tile];
    const int r1 = a.tile_row[tile + 1];
    const long long d0 = static_cast<long long>(tile) * T;
    const long long d1 = d0 + T < total ? d0 + T : total;
    const int e0 = static_cast<int>(d0 - r0);
    const int e1 = static_cast<int>(d1 - r1);
    const int nr = r1 - r0;
    const int ne = e1 - e0;

    // 1. stage row ends and gathered values
    for (int k = tid; k < nr; k += kBlock) s_rowend[k] = a.row_ptr[r0 + 1 + k];
    if (ne > 0) {
      // indices past the tile are clamped to its last edge, so every lane
      // issues its loads without a branch and all of them are in flight
      int j[IPT];
      double v[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const int k = min(i * kBlock + tid, ne - 1);
        j[i] = __builtin_nontemporal_load(a.col + e0 + k);
      }
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const int k = min(i * kBlock + tid, ne - 1);
        v[i] = gather<MODE>(a, j[i], e0 + k);
      }
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const int k = i * kBlock + tid;
        if (k < ne) s_val[k] = v[i];
      }
    }
    const bool head_inc = nr > 0 && a.row_ptr[r0] < e0;
    const bool open = r1 < a.n_rows && e1 > a.row_ptr[r1];
    __syncthreads();

    // 2. this thread's start on the tile's merge path, then its items
    const int len = nr + ne;
    const int diag = tid * IPT < len ? tid * IPT : len;
    int lo = diag - ne > 0 ? diag - ne : 0;
    int hi = diag < nr ? diag : nr;
    while (lo < hi) {
      const int p = (lo + hi) >> 1;
      if (s_rowend[p] <= e0 + diag - p - 1) lo = p + 1; else hi = p;
    }
    const int row_start = lo;
    int row = lo;
    int nz = diag - lo;
    const int dend = diag + IPT < len ? diag + IPT : len;
    double run = 0.0;
    for (int it = diag; it < dend; ++it) {
      if (row < nr && s_rowend[row] <= e0 + nz) {
        s_rowval[row] = run;
        run = 0.0;
        ++row;
      } else {
        run += s_val[nz];
        ++nz;
      }
    }

    // 3. segmented inclusive scan of the carries (rows are non-decreasing in tid)
    s_crow[tid] = row;
    s_cval[tid] = run;
    __syncthreads();
    double v = run;
    for (int off = 1; off < kBlock; off <<= 1) {
      const double add = (tid >= off && s_crow[tid - off] == row) ? s_cval[tid - off] : 0.0;
      __syncthreads();
      v += add;
      s_cval[tid] = v;
      __syncthreads();
    }
    if (row > row_start && tid > 0 && s_crow[tid - 1] == row_start)
      s_rowval[row_start] += s_cval[tid - 1];
    __syncthreads();

    // 4. publish the open row's partial, then the epilogue of the rows that
    //    begin and end here
    if (tid == 0 && open) st_agent(&a.part_open[tile], s_cval[kBlock - 1]);
    for (int k = tid; k < nr; k += kBlock) {
      if (k == 0 && head_inc) continue;
      epilogue<MODE>(a, r0 + k, s_rowval[k], g, sn);
    }
    const double head = s_rowval[0];
    // 5. the row that ended in the previous tile of this block
    if (pend_row >= 0) finish_row<MODE, T>(a, pend_row, pend_tile, pend_head, s_red, g, sn);
    pend_row = head_inc ? r0 : -1;
    pend_tile = tile;
    pend_head = head;
    __syncthreads();  // LDS is refilled by the next tile
  }
  if (pend_row >= 0) finish_row<MODE, T>(a, pend_row, pend_tile, pend_head, s_red, g, sn);

  if constexpr (MODE != kFinal64) {
    // 6. gap: one partial per workgroup, summed in workgroup order by the last
    block_sum2(g, sn, s_red);
    if (tid == 0) {
      st_agent(&a.gap_part[2 * blockIdx.x], g);
      st_agent(&a.gap_part[2 * blockIdx.x + 1], sn);
      const unsigned t = atomicAdd(&a.ctrl->ticket, 1u);
      s_last = t == gridDim.x - 1u;
    }
    __syncthreads();
    if (!s_last) return;
    double G = 0.0, S = 0.0;
    for (int q = tid; q < static_cast<int>(gridDim.x); q += kBlock) {
      G += take_slot(&a.gap_part[2 * q], a.ctrl);
      S += take_slot(&a.gap_part[2 * q + 1], a.ctrl);
    }
    block_sum2(G, S, s_red);
    if (tid == 0) {
      Ctrl* c = a.ctrl;
      c->ticket = 0;
      if (a.gap_out) *a.gap_out = G;
      if (a.count_iter) {
        double gap = G;
        if (c->tol_mode == PSI_TOL_BNORM) gap = G * c->bnorm;
        else if (c->tol_mode == PSI_TOL_REL_L1) gap = S > 0.0 ? G / S : G;
        const int it = c->iter + 1;
        c->iter = it;
        c->gap = gap;
        c->l1 = G;
        c->snorm = S;
        if (a.hist && it - 1 < kHistLen) a.hist[it - 1] = gap;
        if (!isfinite(gap)) {
          c->done = 1;
          c->status = PSI_ENUMERIC;
        } else if (gap <= c->tol) {
          c->done = 1;
          c->status = PSI_OK;
        } else if (it >= c->max_iter) {
          c->done = 1;
          c->status = PSI_ENOTCONV;
        }
      }
    }
  }
}

// Co-resident workgroups for one pass kernel: CUs × workgroups per CU.
template <int IPT, int MODE>
int resident_grid() {
  static int cached = 0;
  if (cached) return cached;
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pass<IPT, MODE>, kBlock, 0) !=
      hipSuccess)
    return 0;
  cached = std::min(kMaxGrid, std::max(1, per_cu) * cus);
  return cached;
}

template <int IPT, int MODE>
psi_status launch_ipt(const PassArgs& a, hipStream_t st) {
  const int cap = resident_grid<IPT, MODE>();
  if (cap <= 0) {
    set_error("could not size the resident grid");
    return PSI_EDEVICE;
  }
  const int grid = std::min(cap, a.n_tiles);
  PassArgs copy = a;
  void* args[] = {&copy};
  PSI_HIP_CHECK(hipLaunchCooperativeKernel(reinterpret_cast<void*>(k_pass<IPT, MODE>), dim3(grid),
                                           dim3(kBlock), args, 0, st));
  return PSI_OK;
}

template <int MODE>
psi_status launch_mode(const PassArgs& a, hipStream_t st) {
  switch (a.tile_items) {
    case 1024: return launch_ipt<4, MODE>(a, st);
    case 1536: return launch_ipt<6, MODE>(a, st);
    case 2048: return launch_ipt<8, MODE>(a, st);
    case 3072: return launch_ipt<12, MODE>(a, st);
    case 4096: return launch_ipt<16, MODE>(a, st);
    default:
      set_error("unsupported tile size " + std::to_string(a.tile_items));
      return PSI_EINVAL;
  }
}

}  // namespace

bool tile_items_supported(int t) {
  return t == 1024 || t == 1536 || t == 2048 || t == 3072 || t == 4096;
}

PassArgs base_args(psi_operator* op) {
  PassArgs a{};
  a.row_ptr = op->row_ptr;
  a.col = op->col;
  a.tile_row = op->tile_row;
  a.n_rows = static_cast<int>(op->n);
  a.n_nnz = static_cast<int>(op->m);
  a.n_tiles = op->n_tiles;
  a.tile_items = op->sched_items;
  a.val64 = op->val64;
  a.c = op->c;
  a.mu = op->mu;
  a.invden = op->invden;
  a.lam = op->lam;
  a.d = op->d;
  a.mu32 = op->mu32;
  a.invden32 = op->invden32;
  a.inv_n = op->n > 0 ? 1.0 / static_cast<double>(op->n) : 0.0;
  a.part_open = op->part_open;
  a.gap_part = op->gap_part;
  a.ctrl = op->ctrl;
  a.hist = op->hist;
  return a;
}

psi_status launch_pass(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t st) {
  (void)op;
  switch (mode) {
    case kStep64: return launch_mode<kStep64>(a, st);
    case kStep64W: return launch_mode<kStep64W>(a, st);
    case kFinal64: return launch_mode<kFinal64>(a, st);
    case kStep32: return launch_mode<kStep32>(a, st);
  }
  set_error("unknown pass mode");
  return PSI_EINVAL;
}

}  // namespace psi
