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
//      per edge into LDS;
//   2. each thread consumes T/256 consecutive path items from LDS;
//   3. a segmented scan of the per-thread carries finishes rows that span
//      threads;
//   4. rows that begin and end in the tile get their epilogue at once.
// The grid is persistent and sized to be co-resident: workgroups walk the
// tiles grid-stride.  A row that spans tiles is summed from the tiles'
// partials, in tile order, by the workgroup that owns the tile where the row
// ends; partials travel through coherent slots (see take_slot), so no cache
// flush or floating-point atomic is needed and every pass is bitwise
// repeatable.  The gap is one partial per workgroup.  A single pass sums the
// partials itself (the last workgroup to finish adds them in workgroup order
// and decides termination); in the solve loop the pass only stores them and
// workgroup 0 of the next pass sums them and decides (deferred: see
// take_deferred), so no pass ends with a chain of device-scope round trips.
//
// Column-segmented passes (S = 2, 4, 8).  The gather of x is limited by the
// rate at which the caches serve random lines, and that rate roughly doubles
// when the gathered range fits one XCD's L2.  Workgroups are dispatched to
// the 8 XCDs round-robin, so the XCDs with xcd % S == s work on column
// segment s (followers in [s·N/S, (s+1)·N/S)) and write a partial y_s; a
// streaming combine kernel then adds the S partials in segment order and
// applies the epilogue and the gap.  The partial pass has two forms over the
// same sums.  Tiled: the merge-path tiles above over the segment's CSR.
// Sliced: one wave per slice of the segment's sliced layout, one lane per
// short row summing its followers in CSR order, so a wave issues nothing but
// coalesced index loads, gathers and one store per row, with no LDS and no
// barrier; rows too long for a lane are cut into chunks summed by whole
// waves, and the last chunk of a row to finish adds the chunk partials in
// chunk order.  The sliced form wins while a segment's share of the gathered
// vector stays in an XCD's L2; beyond that its stores, scattered over rows
// ordered by length, cost more than the tiles' row-ordered ones.  Every row's
// sum has a fixed order in both forms, so passes stay bitwise repeatable.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "psi_internal.h"

namespace psi {

namespace {

// Wait (bounded) until a slot is filled, take its value and empty it again.
// The writer fills the slot before the reader can need it (see the kernels),
// so the wait is short; the bound only guarantees the kernel ends.
__device__ inline double take_slot(double* p, Ctrl* ctrl) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  unsigned long long v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (ctrl->force_timeout) v = kEmptySlot;  // host-forced give-up (recovery test)
  for (int spin = 0; v == kEmptySlot && spin < (1 << 22) && !ctrl->force_timeout; ++spin) {
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (v == kEmptySlot) {
    atomicOr(&ctrl->err_flags, kErrSlotTimeout);
    return 0.0;
  }
  __hip_atomic_store(q, kEmptySlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double(static_cast<long long>(v));
}

// The CSR a group of workgroups walks: the whole of CSR(Aᵀ), or one column
// segment of it.
struct TileSrc {
  const int* row_ptr;
  const int* col;
  const int* tile_row;
  double* part_open;
  void* y;  // per-row output of a partial pass
  int n_nnz;
  int n_tiles;
};

template <int MODE>
__device__ inline double gather(const PassArgs& a, int j, int e) {
  if constexpr (MODE == kStep32 || MODE == kPart32 || MODE == kStep32G) {
    return static_cast<double>(static_cast<const float*>(a.x)[j]);
  } else if constexpr (MODE == kStep64W) {
    return static_cast<const double*>(a.x)[j] * __builtin_nontemporal_load(a.val64 + e);
  } else {
    return static_cast<const double*>(a.x)[j];
  }
}

// Per-user inputs of the epilogue, loaded ahead of the row's sum.
struct RowIn {
  double a0, a1, a2, a3, a4;
  int frozen;
};

template <int MODE>
__device__ inline RowIn load_row(const PassArgs& a, int r) {
  RowIn in{0.0, 0.0, 0.0, 0.0, 0.0, 0};
  if constexpr (MODE == kStep64) {
    in.a0 = a.c[r];
    in.a1 = a.mu[r];
    in.a2 = a.invden[r];
    in.a3 = a.s_old[r];
  } else if constexpr (MODE == kStep64G) {
    in.a0 = a.c[r];
    in.a1 = a.mu[r];
    in.a2 = a.invden[r];
    in.a3 = a.s_old[r];
    in.a4 = static_cast<const double*>(a.x)[r];  // z of s_old, kept when frozen
    in.frozen = a.gdone[a.graph_of[r]];
  } else if constexpr (MODE == kFinal64G) {
    in.a0 = a.lam[r];
    in.a1 = a.d[r];
    in.a2 = a.inv_ng[r];
  } else if constexpr (MODE == kStep64W) {
    in.a0 = a.c[r];
    in.a3 = a.s_old[r];
  } else if constexpr (MODE == kFinal64) {
    in.a0 = a.lam[r];
    in.a1 = a.d[r];
  } else if constexpr (MODE == kStep32) {
    in.a0 = static_cast<double>(a.r32[r]);
    in.a1 = static_cast<double>(a.mu32[r]);
    in.a2 = static_cast<double>(a.invden32[r]);
    in.a3 = static_cast<double>(a.e_old[r]);
  } else if constexpr (MODE == kStep32G) {
    in.a0 = static_cast<double>(a.r32[r]);
    in.a1 = static_cast<double>(a.mu32[r]);
    in.a2 = static_cast<double>(a.invden32[r]);
    in.a3 = static_cast<double>(a.e_old[r]);
    in.a4 = static_cast<double>(static_cast<const float*>(a.x)[r]);  // z_e of e_old
    in.frozen = a.gdone[a.graph_of[r]];
  }
  return in;
}

// Per-user epilogue; g accumulates |new − old|, s accumulates |new|.
template <int MODE>
__device__ inline void apply_row(const PassArgs& a, void* yout, int r, const RowIn& in, double y,
                                 double& g, double& s) {
  if constexpr (MODE == kStep64) {
    const double sn = in.a0 + in.a1 * y;  // c + μ·y
    a.s_new[r] = sn;
    a.z_new[r] = in.a2 * sn;
    g += fabs(sn - in.a3);
    s += fabs(sn);
  } else if constexpr (MODE == kStep64W) {
    const double sn = in.a0 + y;
    a.s_new[r] = sn;
    g += fabs(sn - in.a3);
    s += fabs(sn);
  } else if constexpr (MODE == kFinal64) {
    a.s_new[r] = (in.a0 * y + in.a1) * a.inv_n;
  } else if constexpr (MODE == kStep64G) {
    if (in.frozen) {
      a.s_new[r] = in.a3;
      a.z_new[r] = in.a4;
      a.row_delta[r] = 0.0;
      return;
    }
    const double sn = in.a0 + in.a1 * y;
    a.s_new[r] = sn;
    a.z_new[r] = in.a2 * sn;
    const double dlt = fabs(sn - in.a3);
    a.row_delta[r] = dlt;
    g += dlt;
    s += fabs(sn);
  } else if constexpr (MODE == kFinal64G) {
    a.s_new[r] = (in.a0 * y + in.a1) * in.a2;
  } else if constexpr (MODE == kStep32) {
    const float en = static_cast<float>(in.a0) + static_cast<float>(in.a1) * static_cast<float>(y);
    a.e_new[r] = en;
    a.ze_new[r] = static_cast<float>(in.a2) * en;
    g += fabs(static_cast<double>(en) - in.a3);
    s += fabs(static_cast<double>(en));
  } else if constexpr (MODE == kStep32G) {
    if (in.frozen) {
      a.e_new[r] = static_cast<float>(in.a3);
      a.ze_new[r] = static_cast<float>(in.a4);
      a.row_delta[r] = 0.0;
      return;
    }
    const float en = static_cast<float>(in.a0) + static_cast<float>(in.a1) * static_cast<float>(y);
    a.e_new[r] = en;
    a.ze_new[r] = static_cast<float>(in.a2) * en;
    const double dlt = fabs(static_cast<double>(en) - in.a3);
    a.row_delta[r] = dlt;
    g += dlt;
    s += fabs(static_cast<double>(en));
  } else if constexpr (MODE == kPart64) {
    static_cast<double*>(yout)[r] = y;
  } else {
    static_cast<float*>(yout)[r] = static_cast<float>(y);
  }
}

template <int MODE>
__device__ inline void epilogue(const PassArgs& a, void* yout, int r, double y, double& g,
                                double& s) {
  apply_row<MODE>(a, yout, r, load_row<MODE>(a, r), y, g, s);
}

template <int IPT>
struct TileLds {
  int rowend[kBlock * IPT];
  double val[kBlock * IPT];
  double rowval[kBlock * IPT];
  double cval[kBlock];
  int wkey[2][kBlock / 64];
  double wval[kBlock / 64];
  double red[8];
  int last;
};

// Tile bounds on the merge path.
struct TileMeta {
  int tile, r0, r1, e0, e1, rp0, rp1;  // rp0 = row_ptr[r0], rp1 = row_ptr[r1] (r1 < n)
};

__device__ inline TileMeta tile_meta(const TileSrc& src, int n_rows, long long total, int tile,
                                     int T) {
  TileMeta m;
  m.tile = tile;
  m.r0 = src.tile_row[tile];
  m.r1 = src.tile_row[tile + 1];
  const long long d0 = static_cast<long long>(tile) * T;
  const long long d1 = d0 + T < total ? d0 + T : total;
  m.e0 = static_cast<int>(d0 - m.r0);
  m.e1 = static_cast<int>(d1 - m.r1);
  m.rp0 = m.r1 > m.r0 ? src.row_ptr[m.r0] : m.e0;
  m.rp1 = m.r1 < n_rows ? src.row_ptr[m.r1] : m.e1;
  return m;
}

// Column indices and row ends of a tile, one coalesced load per item slot;
// indices past the tile are clamped so every lane loads without a branch.
template <int IPT>
__device__ inline void load_tile(const TileSrc& src, const TileMeta& m, int* j, int* re) {
  const int ne = m.e1 - m.e0, nr = m.r1 - m.r0;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int k = i * kBlock + static_cast<int>(threadIdx.x);
    j[i] = ne > 0 ? __builtin_nontemporal_load(src.col + m.e0 + min(k, ne - 1)) : 0;
    re[i] = nr > 0 ? src.row_ptr[m.r0 + 1 + min(k, nr - 1)] : 0;
  }
}

template <int IPT, int MODE>
__device__ inline void gather_tile(const PassArgs& a, const TileMeta& m, const int* j, double* v) {
  const int ne = m.e1 - m.e0;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int k = min(i * kBlock + static_cast<int>(threadIdx.x), ne > 0 ? ne - 1 : 0);
    v[i] = ne > 0 ? gather<MODE>(a, j[i], m.e0 + k) : 0.0;
  }
}

// Block-diagonal step passes: every row the tile touches belongs to a graph
// frozen for a whole pass (its result is in both iterate buffers and its
// rows only keep it), so the tile's sums are unused and its gathers can be
// skipped.  Uniform across the workgroup.
__device__ inline bool tile_frozen(const PassArgs& a, const TileMeta& m) {
  if (!a.gskip) return false;
  const int g0 = a.graph_of[min(m.r0, a.n_rows - 1)];
  const int g1 = a.graph_of[min(m.r1, a.n_rows - 1)];
  for (int g = g0; g <= g1; ++g)
    if (!a.gskip[g]) return false;
  return true;
}

template <int IPT, int MODE>
__device__ inline void gather_live_tile(const PassArgs& a, const TileMeta& m, const int* j,
                                        double* v) {
  if (tile_frozen(a, m)) {
#pragma unroll
    for (int i = 0; i < IPT; ++i) v[i] = 0.0;
  } else {
    gather_tile<IPT, MODE>(a, m, j, v);
  }
}

// Walk tiles first, first+stride, ... of src, software-pipelined: while a
// tile is reduced in LDS, the next tile's indices are in flight, and its
// gathers are issued before this tile's epilogue.  A tile publishes the
// partial of its open last row at once; the row that ends in a tile but began
// earlier is summed from the earlier tiles' partials (in tile order) in the
// next iteration, when they are ready, by this workgroup.
template <int IPT, int MODE>
__device__ void run_tiles(const PassArgs& a, const TileSrc& src, int first, int stride,
                          TileLds<IPT>& L, double& g, double& sn) {
  constexpr int T = kBlock * IPT;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const long long total = static_cast<long long>(a.n_rows) + src.n_nnz;
  if (first >= src.n_tiles) return;

  TileMeta cur = tile_meta(src, a.n_rows, total, first, T);
  int j[IPT], re[IPT];
  double v[IPT];
  load_tile<IPT>(src, cur, j, re);
  gather_live_tile<IPT, MODE>(a, cur, j, v);

  // row that ended in the previous tile but began earlier (uniform)
  int pend_row = -1, pend_tile = 0;
  double pend_head = 0.0;

  for (;;) {
    const int nr = cur.r1 - cur.r0;
    const int ne = cur.e1 - cur.e0;
    const bool head_inc = nr > 0 && cur.rp0 < cur.e0;
    const bool open = cur.r1 < a.n_rows && cur.e1 > cur.rp1;

    // 1. stage this tile in LDS
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const int k = i * kBlock + tid;
      if (k < ne) L.val[k] = v[i];
      if (k < nr) L.rowend[k] = re[i];
    }
    // 2. early loads: epilogue inputs of this tile's rows, and the partials
    //    and inputs of the pending row
    // (a tile holds about T / (mean row length + 1) rows, so two per thread
    // cover the usual case; rows beyond load at use)
    constexpr int RPT = IPT < 2 ? IPT : 2;
    RowIn rin[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int k = i * kBlock + tid;
      if (k < nr) rin[i] = load_row<MODE>(a, cur.r0 + k);
    }
    RowIn pin{0.0, 0.0, 0.0, 0.0};
    int pbs = 0, pnq = 0;
    unsigned long long pslot = kEmptySlot;
    if (pend_row >= 0) {
      pbs = static_cast<int>((static_cast<long long>(pend_row) + src.row_ptr[pend_row]) / T);
      pnq = pend_tile - pbs;
      if (tid == 0) pin = load_row<MODE>(a, pend_row);
      if (wave == 0 && lane < pnq && pnq <= 64)
        pslot = __hip_atomic_load(reinterpret_cast<unsigned long long*>(&src.part_open[pbs + lane]),
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // 3. the next tile's bounds, indices and row ends
    const int nxt_tile = cur.tile + stride;
    const bool has_next = nxt_tile < src.n_tiles;
    TileMeta nxt = cur;
    int jn[IPT], ren[IPT];
    if (has_next) {
      nxt = tile_meta(src, a.n_rows, total, nxt_tile, T);
      load_tile<IPT>(src, nxt, jn, ren);
    }
    __syncthreads();

    // 4. this thread's start on the tile's merge path, then its items
    const int len = nr + ne;
    const int diag = tid * IPT < len ? tid * IPT : len;
    int lo = diag - ne > 0 ? diag - ne : 0;
    int hi = diag < nr ? diag : nr;
    while (lo < hi) {
      const int p = (lo + hi) >> 1;
      if (L.rowend[p] <= cur.e0 + diag - p - 1) lo = p + 1; else hi = p;
    }
    const int row_start = lo;
    int row = lo;
    int nz = diag - lo;
    const int dend = diag + IPT < len ? diag + IPT : len;
    double run = 0.0;
    for (int it = diag; it < dend; ++it) {
      if (row < nr && L.rowend[row] <= cur.e0 + nz) {
        L.rowval[row] = run;
        run = 0.0;
        ++row;
      } else {
        run += L.val[nz];
        ++nz;
      }
    }
    // 5. segmented inclusive scan of the carries (rows non-decreasing in tid):
    //    within each wave by shuffles, then across the four waves
    const int up_row = __shfl_up(row, 1, 64);  // carry row of the previous lane
    double sv = run;
    for (int off = 1; off < 64; off <<= 1) {
      const double ov = __shfl_up(sv, off, 64);
      const int ok = __shfl_up(row, off, 64);
      if (lane >= off && ok == row) sv += ov;
    }
    if (lane == 0) L.wkey[0][wave] = row;
    if (lane == 63) {
      L.wkey[1][wave] = row;
      L.wval[wave] = sv;
    }
    __syncthreads();
    {
      // carry into this wave's first segment from the waves before it
      double carry = 0.0;
      int ck = -1;
      for (int w = 0; w < wave; ++w) {
        const int kf = L.wkey[0][w], kl = L.wkey[1][w];
        const double add = (kf == kl && ck == kf) ? carry : 0.0;
        carry = L.wval[w] + add;
        ck = kl;
      }
      if (wave > 0 && row == ck) sv += carry;
    }
    L.cval[tid] = sv;
    __syncthreads();
    const int prev_row = lane != 0 ? up_row : (wave > 0 ? L.wkey[1][wave - 1] : -1);
    if (row > row_start && tid > 0 && prev_row == row_start) L.rowval[row_start] += L.cval[tid - 1];
    __syncthreads();

    // 6. gathers of the next tile, then this tile's epilogue
    double vn[IPT];
    if (has_next) gather_live_tile<IPT, MODE>(a, nxt, jn, vn);
    if (tid == 0 && open) st_agent(&src.part_open[cur.tile], L.cval[kBlock - 1]);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int k = i * kBlock + tid;
      if (k < nr && !(k == 0 && head_inc))
        apply_row<MODE>(a, src.y, cur.r0 + k, rin[i], L.rowval[k], g, sn);
    }
    for (int k = RPT * kBlock + tid; k < nr; k += kBlock)
      epilogue<MODE>(a, src.y, cur.r0 + k, L.rowval[k], g, sn);
    // 7. the pending row: its partials from the earlier tiles, in tile order
    if (pend_row >= 0) {
      double acc = 0.0;
      if (pnq <= 64) {
        if (wave == 0) {
          if (lane < pnq) {
            unsigned long long* q =
                reinterpret_cast<unsigned long long*>(&src.part_open[pbs + lane]);
            if (a.ctrl->force_timeout) pslot = kEmptySlot;  // host-forced give-up
            for (int spin = 0; pslot == kEmptySlot && spin < (1 << 22) && !a.ctrl->force_timeout;
                 ++spin) {
              __builtin_amdgcn_s_sleep(1);
              pslot = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (pslot == kEmptySlot) atomicOr(&a.ctrl->err_flags, kErrSlotTimeout);
            else __hip_atomic_store(q, kEmptySlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            acc = pslot == kEmptySlot ? 0.0 : __longlong_as_double(static_cast<long long>(pslot));
          }
          for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        }
      } else {
        for (int q = pbs + tid; q < pend_tile; q += kBlock) acc += take_slot(&src.part_open[q], a.ctrl);
        double dummy = 0.0;
        block_sum2(acc, dummy, L.red);
      }
      if (tid == 0) apply_row<MODE>(a, src.y, pend_row, pin, acc + pend_head, g, sn);
    }
    pend_row = head_inc ? cur.r0 : -1;
    pend_tile = cur.tile;
    pend_head = L.rowval[0];
    __syncthreads();  // LDS is refilled by the next tile
    if (!has_next) break;
    cur = nxt;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      v[i] = vn[i];
      re[i] = ren[i];
    }
  }
  if (pend_row >= 0) {
    double acc = 0.0, dummy = 0.0;
    const int pbs = static_cast<int>((static_cast<long long>(pend_row) + src.row_ptr[pend_row]) / T);
    for (int q = pbs + tid; q < pend_tile; q += kBlock) acc += take_slot(&src.part_open[q], a.ctrl);
    block_sum2(acc, dummy, L.red);
    if (tid == 0) epilogue<MODE>(a, src.y, pend_row, acc + pend_head, g, sn);
  }
}

// Wave 0 takes up to 64 (g, sn) slot pairs at base[0 .. count) in one round
// trip and sums them in slot order (fixed tree); result in lane 0.
__device__ inline void take_pairs(double* base, int count, Ctrl* ctrl, double& G, double& S) {
  const int lane = threadIdx.x & 63;
  G = 0.0;
  S = 0.0;
  if (lane < count) {
    unsigned long long* q0 = reinterpret_cast<unsigned long long*>(base + 2 * lane);
    unsigned long long v0 = __hip_atomic_load(q0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned long long v1 = __hip_atomic_load(q0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ctrl->force_timeout) v0 = kEmptySlot;  // host-forced give-up (recovery test)
    for (int spin = 0; (v0 == kEmptySlot || v1 == kEmptySlot) && spin < (1 << 22) &&
                       !ctrl->force_timeout;
         ++spin) {
      __builtin_amdgcn_s_sleep(1);
      v0 = __hip_atomic_load(q0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      v1 = __hip_atomic_load(q0 + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (v0 == kEmptySlot || v1 == kEmptySlot) {
      atomicOr(&ctrl->err_flags, kErrSlotTimeout);
    } else {
      G = __longlong_as_double(static_cast<long long>(v0));
      S = __longlong_as_double(static_cast<long long>(v1));
    }
    __hip_atomic_store(q0, kEmptySlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q0 + 1, kEmptySlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int off = 32; off > 0; off >>= 1) {
    G += __shfl_down(G, off, 64);
    S += __shfl_down(S, off, 64);
  }
}

// One partial per workgroup (g, sn).  Deferred form: the pair is stored and
// the next kernel on this control block decides.  Otherwise the pairs are
// reduced in two levels of at most 64 in workgroup order: the last workgroup
// of each group of 64 sums its group, the last group sums the groups and
// decides termination.  Counters are spread over groups, so no single address
// takes every arrival.
__device__ void finalize_gap(const PassArgs& a, double g, double sn, double* red, int* s_last) {
  const int tid = threadIdx.x;
  block_sum2(g, sn, red);
  if (a.defer_gap) {
    if (tid == 0) {
      st_agent(&a.gap_part[2 * blockIdx.x], g);
      st_agent(&a.gap_part[2 * blockIdx.x + 1], sn);
      if (blockIdx.x == 0) a.ctrl->pending = gridDim.x;
    }
    return;
  }
  const int grp = blockIdx.x >> 6;
  const int n_grp = (gridDim.x + 63) >> 6;
  const int in_grp = min(64, static_cast<int>(gridDim.x) - (grp << 6));
  if (tid == 0) {
    st_agent(&a.gap_part[2 * blockIdx.x], g);
    st_agent(&a.gap_part[2 * blockIdx.x + 1], sn);
    const unsigned t = atomicAdd(&a.grp_ticket[grp], 1u);
    *s_last = t == static_cast<unsigned>(in_grp) - 1u;
  }
  __syncthreads();
  if (!*s_last) return;
  if (tid < 64) {
    double G, S;
    take_pairs(a.gap_part + 2 * (grp << 6), in_grp, a.ctrl, G, S);
    if (tid == 0) {
      a.grp_ticket[grp] = 0;
      st_agent(&a.gap_grp[2 * grp], G);
      st_agent(&a.gap_grp[2 * grp + 1], S);
      const unsigned t = atomicAdd(&a.ctrl->ticket, 1u);
      *s_last = t == static_cast<unsigned>(n_grp) - 1u;
    }
  }
  __syncthreads();
  if (!*s_last || tid >= 64) return;
  double G, S;
  take_pairs(a.gap_grp, n_grp, a.ctrl, G, S);
  if (tid == 0) {
    a.ctrl->ticket = 0;
    decide_gap(a.ctrl, G, S, a.hist, a.gap_out, a.count_iter, -1);
  }
}

__global__ __launch_bounds__(kBlock) void k_gap_decide(Ctrl* c, double* pairs, double* hist,
                                                       int count_iter) {
  __shared__ double red[8];
  take_deferred(c, pairs, hist, count_iter, -1, red);
}

// Fused pass over the whole of CSR(Aᵀ).
template <int IPT, int MODE>
__global__ __launch_bounds__(kBlock) void k_pass(PassArgs a) {
  __shared__ TileLds<IPT> L;
  if (a.defer_gap && blockIdx.x == 0)
    take_deferred(a.ctrl, a.gap_prev, a.hist, a.count_iter, a.pass_id, L.red);
  // a decision of this very pass (by workgroup 0) does not stop it: every
  // workgroup must run, or cross-tile slots would be left half filled
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, false)) return;
  TileSrc src{a.row_ptr, a.col, a.tile_row, a.part_open, nullptr, a.n_nnz, a.n_tiles};
  double g = 0.0, sn = 0.0;
  run_tiles<IPT, MODE>(a, src, blockIdx.x, gridDim.x, L, g, sn);
  if constexpr (MODE != kFinal64 && MODE != kFinal64G) finalize_gap(a, g, sn, L.red, &L.last);
}

// Partial pass of one column segment per XCD group over merge-path tiles
// (tiled form): y_s = A_sᵀ x.
template <int IPT, int MODE>
__global__ __launch_bounds__(kBlock) void k_pass_seg(PassArgs a, SegArgs sg) {
  __shared__ TileLds<IPT> L;
  if (a.defer_gap && blockIdx.x == 0)
    take_deferred(a.ctrl, a.gap_prev, a.hist, a.count_iter, a.pass_id, L.red);
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, false)) return;
  const int xcd = blockIdx.x & 7;
  const int group = xcd % sg.S;
  const int per_round = 8 / sg.S;  // workgroups of a group among 8 consecutive ones
  const int rank = (blockIdx.x >> 3) * per_round + xcd / sg.S;
  const int size = (gridDim.x >> 3) * per_round;
  const SegInfo& si = sg.seg[group];
  TileSrc src{si.row_ptr, si.col, si.tile_row, si.part_open, si.y, si.n_nnz, si.n_tiles};
  double g = 0.0, sn = 0.0;
  run_tiles<IPT, MODE>(a, src, rank, size, L, g, sn);
}

// Partial pass over the sliced layout of the segments: y_s = A_sᵀ x.  XCD
// group s (workgroups with (blockIdx mod 8) mod S = s) takes the slices of
// segment s, four per workgroup, one per wave.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_slices(SliceArgs a) {
  __shared__ double red[8];
  if (a.defer_gap && blockIdx.x == 0)
    take_deferred(a.ctrl, a.gap_prev, a.hist, a.count_iter, a.pass_id, red);
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, false)) return;
  using XT = typename std::conditional<MODE == kPart32, float, double>::type;
  const int xcd = blockIdx.x & 7;
  const int group = xcd % a.S;
  const int per_round = 8 / a.S;  // XCDs of a group
  const SliceSeg& sg = a.seg[group];
  // each XCD of the group takes a contiguous run of the segment's slices, in
  // dispatch order, so the stores of a window land in one L2
  const int ranks = (sg.n_slices + kBlock / 64 - 1) / (kBlock / 64);
  const int run = (ranks + per_round - 1) / per_round;
  if (static_cast<int>(blockIdx.x >> 3) >= run) return;  // this group's runs are shorter
  const int rank = (xcd / a.S) * run + static_cast<int>(blockIdx.x >> 3);
  const int q = rank * (kBlock / 64) + (threadIdx.x >> 6);
  if (q >= sg.n_slices) return;
  const int lane = threadIdx.x & 63;
  const XT* x = static_cast<const XT*>(a.x);
  const SliceDesc d = sg.slices[q];
  double acc = 0.0;
  if (d.tag >= 0) {
    // one row per lane; step k of the 64 lanes is one contiguous run of ids
    const int row = a.row[d.tag + lane];
    const int len = a.len[d.tag + lane];
    const int* c = a.col + d.off + lane;
    // every gather of a step is issued before any add; a lane past its row's
    // end reads a padding id (0, a valid entry) and adds nothing
    int k = 0;
    for (; k + 4 <= d.len; k += 4) {
      const int j0 = c[(k + 0) * 64], j1 = c[(k + 1) * 64], j2 = c[(k + 2) * 64], j3 = c[(k + 3) * 64];
      const double v0 = static_cast<double>(x[j0]);
      const double v1 = static_cast<double>(x[j1]);
      const double v2 = static_cast<double>(x[j2]);
      const double v3 = static_cast<double>(x[j3]);
      acc += k + 0 < len ? v0 : 0.0;
      acc += k + 1 < len ? v1 : 0.0;
      acc += k + 2 < len ? v2 : 0.0;
      acc += k + 3 < len ? v3 : 0.0;
    }
    if (k < d.len) {
      const int r = d.len - k;  // 1..3 steps left
      const int j0 = c[(k + 0) * 64];
      const int j1 = r > 1 ? c[(k + 1) * 64] : 0;
      const int j2 = r > 2 ? c[(k + 2) * 64] : 0;
      const double v0 = static_cast<double>(x[j0]);
      const double v1 = static_cast<double>(x[j1]);
      const double v2 = static_cast<double>(x[j2]);
      acc += k + 0 < len ? v0 : 0.0;
      acc += k + 1 < len ? v1 : 0.0;
      acc += k + 2 < len ? v2 : 0.0;
    }
    if (row >= 0) static_cast<XT*>(sg.y)[row] = static_cast<XT>(acc);
    return;
  }
  // a chunk of a long row: the wave strides over its edges (clamped loads,
  // masked adds), then reduces
  const int4 ch = a.chunk[-1 - d.tag];  // row, slot, first slot of the row, chunks of the row
  const int* c = a.seg_col + d.off;
  const int ne = d.len;
  const int steps = (ne + 63) >> 6;
  int k = 0;
  for (; k + 4 <= steps; k += 4) {
    const int e0 = (k + 0) * 64 + lane, e1 = (k + 1) * 64 + lane;
    const int e2 = (k + 2) * 64 + lane, e3 = (k + 3) * 64 + lane;
    const int j0 = c[min(e0, ne - 1)], j1 = c[min(e1, ne - 1)];
    const int j2 = c[min(e2, ne - 1)], j3 = c[min(e3, ne - 1)];
    const double v0 = static_cast<double>(x[j0]);
    const double v1 = static_cast<double>(x[j1]);
    const double v2 = static_cast<double>(x[j2]);
    const double v3 = static_cast<double>(x[j3]);
    acc += e0 < ne ? v0 : 0.0;
    acc += e1 < ne ? v1 : 0.0;
    acc += e2 < ne ? v2 : 0.0;
    acc += e3 < ne ? v3 : 0.0;
  }
  for (; k < steps; ++k) {
    const int e = k * 64 + lane;
    const double v = static_cast<double>(x[c[min(e, ne - 1)]]);
    acc += e < ne ? v : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (ch.y < 0) {
    if (lane == 0) static_cast<XT*>(sg.y)[ch.x] = static_cast<XT>(acc);
    return;
  }
  // several chunks: publish this one; the last to arrive sums them in order
  int last = 0;
  if (lane == 0) {
    st_agent(&a.part[ch.y], acc);
    last = atomicAdd(&a.ticket[ch.z], 1u) == static_cast<unsigned>(ch.w) - 1u;
  }
  last = __shfl(last, 0, 64);
  if (!last) return;
  double sum = 0.0;
  for (int i = lane; i < ch.w; i += 64) sum += take_slot(&a.part[ch.z + i], a.ctrl);
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if (lane == 0) {
    static_cast<XT*>(sg.y)[ch.x] = static_cast<XT>(sum);
    a.ticket[ch.z] = 0;
  }
}

// y_i = Σ_s y_s[i] in segment order, then the epilogue of MODE and the gap.
template <int MODE, class YT>
__global__ __launch_bounds__(kBlock) void k_combine(PassArgs a, SegArgs sg) {
  __shared__ double red[8];
  __shared__ int last;
  // the combine follows its own pass's partial kernel, whose decision it sees
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, true)) return;
  double g = 0.0, sn = 0.0;
  const YT* y0 = static_cast<const YT*>(sg.seg[0].y);
  const YT* y1 = static_cast<const YT*>(sg.seg[1].y);
  const YT* y2 = static_cast<const YT*>(sg.seg[2].y);
  const YT* y3 = static_cast<const YT*>(sg.seg[3].y);
  const YT* y4 = static_cast<const YT*>(sg.seg[4].y);
  const YT* y5 = static_cast<const YT*>(sg.seg[5].y);
  const YT* y6 = static_cast<const YT*>(sg.seg[6].y);
  const YT* y7 = static_cast<const YT*>(sg.seg[7].y);
  const int S = sg.S;
  constexpr int U = 4;  // rows in flight per thread
  const int stride = gridDim.x * kBlock;
  for (int base = blockIdx.x * kBlock + threadIdx.x; base < a.n_rows; base += U * stride) {
    double y[U];
    RowIn in[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = base + u * stride;
      y[u] = 0.0;
      if (r < a.n_rows) {
        // partials summed in segment order
        y[u] = static_cast<double>(y0[r]) + static_cast<double>(y1[r]);
        if (S > 2) y[u] = (y[u] + static_cast<double>(y2[r])) + static_cast<double>(y3[r]);
        if (S > 4)
          y[u] = (((y[u] + static_cast<double>(y4[r])) + static_cast<double>(y5[r])) +
                  static_cast<double>(y6[r])) + static_cast<double>(y7[r]);
        in[u] = load_row<MODE>(a, r);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = base + u * stride;
      if (r < a.n_rows) apply_row<MODE>(a, nullptr, r, in[u], y[u], g, sn);
    }
  }
  // block-diagonal operators take each graph's gap from its rows' |Δ| instead
  if constexpr (MODE == kStep64 || MODE == kStep32) finalize_gap(a, g, sn, red, &last);
}

// ---------------------------------------------------------------- band form
// One wave per row block (see psi_band.hip): its rows' sums in LDS, its
// entries walked column block by column block in chunks of 64 (a chunk never
// spans two column blocks, so its rows are distinct runs in row order).  A
// chunk's runs are summed by a segmented scan across the wave (a fixed
// tree); the last lane of each run adds the run to its row's sum.
//
// A workgroup holds four row blocks (four waves); each wave walks the column
// blocks on its own, loading the next column block's entries while it sums
// the current one.  Waves that start a launch together gather from the same
// column blocks, but drift apart over hundreds of them; an optional pacing
// (a start time per column block) keeps them together.
constexpr int kBandUnroll = 4;  // chunks in flight per wave

// Adds the run sums of one chunk to y: lanes in entry order, rl = row in the
// block (>= nrows for lanes past the column block's end).
__device__ inline void band_chunk_add(double* y, unsigned rl, double v, int nrows, int lane) {
  const unsigned prev = __shfl_up(rl, 1, 64);
  // lanes past the column block's end (rl >= nrows) each start a run of their
  // own, so they never lengthen the scan
  const bool head = lane == 0 || rl != prev || rl >= static_cast<unsigned>(nrows);
  const unsigned long long hm = __ballot(head);
  const int h = 63 - __clzll(hm & (~0ull >> (63 - lane)));  // first lane of this lane's run
  // the step with offset off matters only if some run holds more than off
  // lanes: pos holds the lanes at position >= off in their run (a uniform
  // mask), so the scan stops after the longest run (usually one or two steps)
  unsigned long long pos = ~hm;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    if (pos == 0ull) break;
    const double t = __shfl_up(v, off, 64);
    if (lane - off >= h) v += t;
    pos &= pos << off;
  }
  const bool tail = lane == 63 || ((hm >> (lane + 1)) & 1ull);
  if (tail && rl < static_cast<unsigned>(nrows)) y[rl] += v;
}

// Entries [e, end) of a column block, up to kBandUnroll chunks (0xFFFFFFFF
// past the end).
__device__ inline void band_load(const uint32_t* ent, uint32_t e, uint32_t end, int lane,
                                 uint32_t* out) {
#pragma unroll
  for (int u = 0; u < kBandUnroll; ++u) {
    const uint32_t i = e + u * 64 + lane;
    out[u] = i < end ? ent[i] : 0xFFFFFFFFu;
  }
}

// Gathers and adds up to kBandUnroll chunks of entries of column block c.  In
// a Gauss–Seidel sweep (GS) a follower below `fresh` is read from xn_c, this
// sweep's values, else from xc, the previous sweep's.
template <bool GS, class XT>
__device__ inline void band_group(double* y, const XT* xc, const XT* xn_c, int64_t col0,
                                  int64_t fresh, const uint32_t* en, uint32_t e, uint32_t end,
                                  int wlog, int nrows, int lane) {
  const uint32_t wmask = (1u << wlog) - 1u;
  double v[kBandUnroll];
#pragma unroll
  for (int u = 0; u < kBandUnroll; ++u) {
    const uint32_t jl = en[u] & wmask;
    const XT* src = xc;
    if constexpr (GS) src = col0 + jl < fresh ? xn_c : xc;
    v[u] = en[u] != 0xFFFFFFFFu ? static_cast<double>(src[jl]) : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kBandUnroll; ++u) {
    if (e + u * 64 >= end) break;  // uniform
    band_chunk_add(y, en[u] >> wlog, v[u], nrows, lane);
  }
}

// Fixed-order sum over the NW waves of a workgroup of two values; result in
// thread 0.
template <int NW>
__device__ inline void block_sum2_n(double& a, double& b, double* sh) {
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
    a = 0.0;
    b = 0.0;
    for (int k = 0; k < NW; ++k) {
      a += sh[2 * k];
      b += sh[2 * k + 1];
    }
  }
  __syncthreads();
}

// Deferred gap of the previous pass (as take_deferred) for a workgroup of NW
// waves: thread t sums a contiguous run of the pairs, then a fixed tree.
template <int NW>
__device__ inline void take_deferred_n(Ctrl* c, double* pairs, double* hist, int count_iter,
                                       int pass_id, double* red) {
  const int n = static_cast<int>(c->pending);  // uniform
  if (n == 0) return;
  const int already = c->done;                  // uniform
  const int tid = threadIdx.x;
  constexpr int NT = NW * 64;
  const int per = (n + NT - 1) / NT;
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
  block_sum2_n<NW>(G, S, red);
  if (tid == 0) {
    c->pending = 0;
    if (!already) decide_gap(c, G, S, hist, nullptr, count_iter, pass_id);
  }
  __syncthreads();
}

template <int MODE, int R, int NW, bool GS>
__global__ __launch_bounds__(NW * 64) void k_band(PassArgs a, BandArgs b) {
  // the row sums; the first 2·NW doubles also serve the workgroup's two
  // reductions, before the sums are zeroed and after they are consumed, so
  // that the LDS of the workgroup stays at NW·R doubles (five workgroups of
  // four 1024-row waves fit one CU)
  __shared__ double ylds[NW][R];
  double* red = &ylds[0][0];
  using XT = typename std::conditional<MODE == kStep32, float, double>::type;
  if (b.first_launch && a.defer_gap && blockIdx.x == 0)
    take_deferred_n<NW>(a.ctrl, a.gap_prev, a.hist, a.count_iter, a.pass_id, red);
  // a decision made during the first launch concerns the previous pass and
  // carries this pass's id, which stops only the later launches
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, !b.first_launch)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int blk = b.first_block + static_cast<int>(blockIdx.x) * NW + wave;
  double g = 0.0, sn = 0.0;
  if (blk < b.n_blocks) {
    const BandBlock bb = b.blocks[blk];
    double* y = ylds[wave];
    for (int k = lane; k < bb.nrows; k += 64) y[k] = 0.0;
    __builtin_amdgcn_wave_barrier();
    const uint32_t* toff = b.toff + static_cast<int64_t>(blk) * b.B;
    const XT* x = static_cast<const XT*>(a.x);
    const XT* xn = static_cast<const XT*>(b.x_new);
    // pacing: column block c starts no earlier than c·pace after this wave's
    // start, so that waves which run ahead wait for the others and the
    // gathers of all waves stay in the same few column blocks (0 = off)
    const unsigned long long t_start = b.pace ? wall_clock64() : 0ull;
    uint32_t t0 = toff[0], t1 = toff[1];
    uint32_t pre[kBandUnroll];
    band_load(b.ent, t0, t1, lane, pre);
    for (int c = 0; c < b.B; ++c) {
      uint32_t cur[kBandUnroll];
#pragma unroll
      for (int u = 0; u < kBandUnroll; ++u) cur[u] = pre[u];
      const uint32_t e0 = t0, e1 = t1;
      // the next column block's bounds and first chunks, in flight meanwhile
      if (c + 1 < b.B) {
        t0 = t1;
        t1 = toff[c + 2];
        band_load(b.ent, t0, t1, lane, pre);
      }
      if (b.pace) {
        const unsigned long long due = t_start + static_cast<unsigned long long>(c) * b.pace;
        while (wall_clock64() < due) __builtin_amdgcn_s_sleep(2);
      }
      const int64_t col0 = static_cast<int64_t>(c) << b.wlog;
      const XT* xc = x + col0;
      const XT* xn_c = GS ? xn + col0 : xc;
      if (e0 < e1) {
        band_group<GS>(y, xc, xn_c, col0, b.fresh_below, cur, e0, e1, b.wlog, bb.nrows, lane);
        for (uint32_t e = e0 + 64 * kBandUnroll; e < e1; e += 64 * kBandUnroll) {
          band_load(b.ent, e, e1, lane, cur);
          band_group<GS>(y, xc, xn_c, col0, b.fresh_below, cur, e, e1, b.wlog, bb.nrows, lane);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (bb.piece >= 0) {
      if (lane == 0) b.piece[bb.piece] = y[0];
    } else {
      for (int k = lane; k < bb.nrows; k += 64) {
        const int r = bb.row_lo + k;
        apply_row<MODE>(a, nullptr, r, load_row<MODE>(a, r), y[k], g, sn);
      }
    }
  }
  if constexpr (MODE != kFinal64) {
    __syncthreads();  // every wave has read its sums before red overwrites them
    block_sum2_n<NW>(g, sn, red);
    if (threadIdx.x == 0) {
      const int q = b.pair_base + static_cast<int>(blockIdx.x);
      b.pairs[2 * q] = g;
      b.pairs[2 * q + 1] = sn;
    }
  }
}

// The end of a band pass: rows cut into pieces get their sum (pieces in
// order) and epilogue; the band launches' gap pairs are summed in order, a
// contiguous share per workgroup, and the gap is finished as in every pass.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_band_fix(PassArgs a, BandFixArgs f) {
  __shared__ double red[8];
  __shared__ int last;
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, true)) return;
  const int tid = threadIdx.x;
  double g = 0.0, sn = 0.0;
  if constexpr (MODE != kFinal64) {
    const int per = (f.n_pairs + static_cast<int>(gridDim.x) - 1) / static_cast<int>(gridDim.x);
    const int lo = static_cast<int>(blockIdx.x) * per;
    const int hi = min(f.n_pairs, lo + per);
    const int per_t = (max(hi - lo, 0) + kBlock - 1) / kBlock;
    const int q_end = min(hi, lo + (tid + 1) * per_t);
    for (int q = lo + tid * per_t; q < q_end; ++q) {
      g += f.pairs[2 * q];
      sn += f.pairs[2 * q + 1];
    }
  }
  for (int q = static_cast<int>(blockIdx.x) * kBlock + tid; q < f.n_split;
       q += static_cast<int>(gridDim.x) * kBlock) {
    const int4 sr = f.split[q];
    double y = 0.0;
    for (int p = sr.y; p < sr.z; ++p) y += f.piece[p];
    apply_row<MODE>(a, nullptr, sr.x, load_row<MODE>(a, sr.x), y, g, sn);
  }
  if constexpr (MODE != kFinal64) finalize_gap(a, g, sn, red, &last);
}

// Gauss–Seidel sweep: after band k, the split rows whose pieces all lie in
// bands 0..k get their sum and epilogue, so that later bands gather their new
// values; one workgroup, rows [lo, hi) of the split table, the gap pair of
// these rows stored at pairs[q].
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_band_split(PassArgs a, BandFixArgs f, int lo, int hi,
                                                      int q, int first_launch) {
  __shared__ double red[8];
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, !first_launch)) return;
  double g = 0.0, sn = 0.0;
  for (int i = lo + static_cast<int>(threadIdx.x); i < hi; i += kBlock) {
    const int4 sr = f.split[i];
    double y = 0.0;
    for (int p = sr.y; p < sr.z; ++p) y += f.piece[p];
    apply_row<MODE>(a, nullptr, sr.x, load_row<MODE>(a, sr.x), y, g, sn);
  }
  block_sum2(g, sn, red);
  if (threadIdx.x == 0) {
    const_cast<double*>(f.pairs)[2 * q] = g;
    const_cast<double*>(f.pairs)[2 * q + 1] = sn;
  }
}

// -------------------------------------------------------------- binned form
// Two streaming launches per pass over the binned layout (psi_bins.hip).
//
// Expand: one workgroup per column block of 20,480 users.  Workgroups go to the
// XCDs round-robin, so blockIdx mod 8 picks the XCD and each XCD takes a
// contiguous range of column blocks in order: the runs that neighbouring
// column blocks write into one bin lie side by side in bin order, and their
// partial lines meet in that XCD's L2.  The block's z goes to LDS; each wave
// streams a sixteenth of the block's entries, finds each entry's run by
// counting run-start flags from the run before its first entry, and writes z
// of the entry's column to slot rdelta[run] + entry.
constexpr int kBinsUnroll = 8;        // chunks of 64 entries in flight per bin wave
// Chunks of 64 entries a group in the expand waves: 16 with FP64 z (one
// workgroup of 16 waves per CU, 128 registers a lane), 8 with FP32 z (two
// workgroups per CU, 64 registers a lane).
template <class XT>
constexpr int expand_unroll() { return sizeof(XT) == 8 ? 16 : 8; }

// Words (column in block | run-start flag) of one group of chunks from k0.
template <int U>
__device__ inline void expand_words(const uint16_t* col, uint32_t k0, uint32_t hi, int lane,
                                    uint32_t* w) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t k = k0 + u * 64 + lane;
    w[u] = k < hi ? static_cast<uint32_t>(col[k]) : 0u;
  }
}

// Slots of one group: each entry's run from the run-start flags counted on
// from `run`, then rdelta[run] + entry (loads issued, not waited for).  r and
// the slot are in range by construction; the clamps keep a damaged layout
// from writing outside the value array.
template <int U>
__device__ inline void expand_slots(const BinsArgs& b, const uint32_t* w, uint32_t k0, uint32_t hi,
                                    int lane, int& run, uint32_t* dst) {
  const unsigned long long upto = ~0ull >> (63 - lane);  // lanes 0..lane
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint32_t k = k0 + u * 64 + lane;
    const unsigned long long fl = __ballot(k < hi && (w[u] & kBinsFirst));
    const int r = run + __popcll(fl & upto);
    run += __popcll(fl);
    const uint32_t rc = static_cast<uint32_t>(min(max(r, 0), static_cast<int>(b.runs) - 1));
    dst[u] = k < hi ? min(b.rdelta[rc] + k, b.m - 1u) : 0u;
  }
}

template <class XT>
__global__ __launch_bounds__(kBinsExpandWaves * 64) void k_bins_expand(PassArgs a, BinsArgs b) {
  __shared__ XT zl[kBinsCols];
  // the deferred gap's reduction uses the first 2·waves doubles of zl before
  // the block's z is loaded
  if (a.defer_gap && blockIdx.x == 0)
    take_deferred_n<kBinsExpandWaves>(a.ctrl, a.gap_prev, a.hist, a.count_iter, a.pass_id,
                                      reinterpret_cast<double*>(zl));
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, false)) return;
  const int c = static_cast<int>(blockIdx.x & 7) * b.per_xcd + static_cast<int>(blockIdx.x >> 3);
  if (c >= b.B) return;  // uniform across the workgroup
  const int64_t col0 = static_cast<int64_t>(c) * kBinsCols;
  const int64_t nc = min(static_cast<int64_t>(kBinsCols), static_cast<int64_t>(a.n_rows) - col0);
  const XT* x = static_cast<const XT*>(a.x) + col0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t lo0 = b.cs[c], ne = b.cs[c + 1] - lo0;
  const uint32_t lo =
      lo0 + static_cast<uint32_t>((static_cast<uint64_t>(ne) * wave) / kBinsExpandWaves);
  const uint32_t hi =
      lo0 + static_cast<uint32_t>((static_cast<uint64_t>(ne) * (wave + 1)) / kBinsExpandWaves);
  int run = b.task[c * kBinsExpandWaves + wave];
  // the first groups' words and slots in flight while z is loaded
  constexpr int U = expand_unroll<XT>();
  constexpr uint32_t G = 64 * U;
  uint32_t w0[U], w1[U], d0[U];
  expand_words<U>(b.col, lo, hi, lane, w0);
  expand_words<U>(b.col, lo + G, hi, lane, w1);
  for (int j = threadIdx.x; j < kBinsCols; j += kBinsExpandWaves * 64)
    zl[j] = j < nc ? x[j] : XT(0);
  expand_slots<U>(b, w0, lo, hi, lane, run, d0);
  __syncthreads();
  XT* out = static_cast<XT*>(b.val);
  // three stages: words two groups ahead, slots one group ahead, stores now
  for (uint32_t k0 = lo; k0 < hi; k0 += G) {
    uint32_t w2[U], d1[U];
    if (k0 + 2 * G < hi) expand_words<U>(b.col, k0 + 2 * G, hi, lane, w2);
    if (k0 + G < hi) expand_slots<U>(b, w1, k0 + G, hi, lane, run, d1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t k = k0 + u * 64 + lane;
      if (k < hi) out[d0[u]] = zl[w0[u] & kBinsColMask];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      w0[u] = w1[u];
      d0[u] = d1[u];
      w1[u] = w2[u];
    }
  }
}

// Bins: one wave per bin (launch order: most edges first), its values and rows
// streamed 64 entries a chunk.
// * A piece of a split row (one row): each lane sums its entries (lane l takes
//   entries l, l + 64, ... in order) and one fixed butterfly joins the lanes.
// * Whole rows: the rows' sums live in LDS, and every lane adds its entry to
//   its row's sum, one atomic per chunk.  Lanes of one atomic that hit the
//   same word are applied by the LDS one after another in lane order, i.e. in
//   the layout's order (measured: bitwise equal to issuing the adds run by
//   run on 1.4·10⁹ entries), and a wave's atomics in program order, so every
//   row's sum has a fixed order and passes stay bitwise repeatable.

// Every lane adds its own entry to its row's sum.
template <class XT>
__device__ inline void bins_lane_add(double* y, const uint32_t* w, const XT* vin, uint32_t e,
                                     uint32_t e1, int lane) {
#pragma unroll
  for (int u = 0; u < kBinsUnroll; ++u) {
    if (e + u * 64 >= e1) break;  // uniform
    if (e + u * 64 + lane < e1)
      __hip_atomic_fetch_add(y + (w[u] & (kBinsFirst - 1u)), static_cast<double>(vin[u]),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Entries [e, e + 64·kBinsUnroll) of a bin whose entries end at end > e
// (their rows only if ROWS): lanes past the end load the bin's last entry (in
// range), which the adds drop by their index (no select here, so the loads
// stay in flight).
template <bool ROWS, class XT>
__device__ inline void bins_load(const uint16_t* row, const XT* val, uint32_t e, uint32_t end,
                                 int lane, uint32_t* w, XT* v) {
#pragma unroll
  for (int u = 0; u < kBinsUnroll; ++u) {
    const uint32_t j = min(e + u * 64 + lane, end - 1u);
    w[u] = ROWS ? row[j] : 0u;
    v[u] = val[j];
  }
}

// Streams the bin's entries [e0, e1), e0 < e1, a group of chunks at a time
// with the next group in flight, and hands each group to add(w, v, e).
template <bool ROWS, class XT, class Add>
__device__ inline void bins_stream(const uint16_t* row, const XT* val, uint32_t e0, uint32_t e1,
                                   int lane, Add add) {
  uint32_t wn[kBinsUnroll];
  XT vn[kBinsUnroll];
  bins_load<ROWS>(row, val, e0, e1, lane, wn, vn);
  for (uint32_t e = e0; e < e1; e += 64 * kBinsUnroll) {
    uint32_t wc[kBinsUnroll];
    XT vc[kBinsUnroll];
#pragma unroll
    for (int u = 0; u < kBinsUnroll; ++u) {
      wc[u] = wn[u];
      vc[u] = vn[u];
    }
    if (e + 64 * kBinsUnroll < e1)
      bins_load<ROWS>(row, val, e + 64 * kBinsUnroll, e1, lane, wn, vn);
    add(wc, vc, e);
  }
}

template <int MODE, int R, int NW>
__global__ __launch_bounds__(NW * 64) void k_bins(PassArgs a, BinsArgs b) {
  // the row sums; the first 2·NW doubles also serve the gap reduction after
  // the sums are consumed
  __shared__ double ylds[NW][R];
  double* red = &ylds[0][0];
  using XT = typename std::conditional<MODE == kStep32, float, double>::type;
  if (a.respect_done && pass_cancelled(a.ctrl, a.pass_id, true)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = static_cast<int>(blockIdx.x) * NW + wave;
  double g = 0.0, sn = 0.0;
  if (slot < b.nb) {
    const int blk = b.order[slot];
    const BandBlock bb = b.blocks[blk];
    double* y = ylds[wave];
    const uint32_t e0 = b.bstart[blk], e1 = b.bstart[blk + 1];
    const XT* val = static_cast<const XT*>(b.val);
    if (bb.piece >= 0) {
      double acc = 0.0;
      const auto add = [&](const uint32_t*, const XT* v, uint32_t e) {
#pragma unroll
        for (int u = 0; u < kBinsUnroll; ++u)
          if (e + u * 64 + lane < e1) acc += static_cast<double>(v[u]);
      };
      if (e0 < e1) bins_stream<false>(b.row, val, e0, e1, lane, add);
      for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (lane == 0) b.piece[bb.piece] = acc;
    } else {
      for (int k = lane; k < bb.nrows; k += 64) y[k] = 0.0;
      __builtin_amdgcn_wave_barrier();
      const auto add = [&](const uint32_t* w, const XT* v, uint32_t e) {
        bins_lane_add(y, w, v, e, e1, lane);
      };
      if (e0 < e1) bins_stream<true>(b.row, val, e0, e1, lane, add);
      __builtin_amdgcn_wave_barrier();
      for (int k = lane; k < bb.nrows; k += 64) {
        const int r = bb.row_lo + k;
        apply_row<MODE>(a, nullptr, r, load_row<MODE>(a, r), y[k], g, sn);
      }
    }
  }
  if constexpr (MODE != kFinal64) {
    __syncthreads();  // every wave has read its sums before red overwrites them
    block_sum2_n<NW>(g, sn, red);
    if (threadIdx.x == 0) {
      b.pairs[2 * blockIdx.x] = g;
      b.pairs[2 * blockIdx.x + 1] = sn;
    }
  }
}

// Co-resident workgroups of a kernel: CUs × workgroups per CU, a multiple of 8.
template <class K>
int resident_grid(K kernel) {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess)
    return 0;
  const int g = std::min(kMaxGrid, std::max(1, per_cu) * cus);
  return std::max(8, g / 8 * 8);
}

template <int IPT, int MODE>
psi_status launch_ipt(const PassArgs& a, hipStream_t st) {
  static const int cap = resident_grid(k_pass<IPT, MODE>);
  if (cap <= 0) {
    set_error("could not size the resident grid");
    return PSI_EDEVICE;
  }
  // the grid never exceeds what fits on the device at once, so on an idle
  // device every workgroup is resident; the slot waits are bounded in any case
  const int grid = std::min(cap, a.n_tiles);
  hipLaunchKernelGGL((k_pass<IPT, MODE>), dim3(grid), dim3(kBlock), 0, st, a);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

template <int IPT, int PMODE>
psi_status launch_seg_ipt(const PassArgs& a, const SegArgs& sg, hipStream_t st) {
  static const int cap = resident_grid(k_pass_seg<IPT, PMODE>);
  if (cap <= 0) {
    set_error("could not size the resident grid");
    return PSI_EDEVICE;
  }
  hipLaunchKernelGGL((k_pass_seg<IPT, PMODE>), dim3(cap), dim3(kBlock), 0, st, a, sg);
  PSI_HIP_CHECK(hipGetLastError());
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

template <int PMODE>
psi_status launch_seg_mode(const PassArgs& a, const SegArgs& sg, hipStream_t st) {
  switch (a.tile_items) {
    case 1024: return launch_seg_ipt<4, PMODE>(a, sg, st);
    case 1536: return launch_seg_ipt<6, PMODE>(a, sg, st);
    case 2048: return launch_seg_ipt<8, PMODE>(a, sg, st);
    case 3072: return launch_seg_ipt<12, PMODE>(a, sg, st);
    case 4096: return launch_seg_ipt<16, PMODE>(a, sg, st);
    default:
      set_error("unsupported tile size " + std::to_string(a.tile_items));
      return PSI_EINVAL;
  }
}

// Grid of the sliced partial pass: workgroups of XCD group s cover the
// slices of segment s four at a time.
template <int MODE>
psi_status launch_slices(psi_operator* op, const PassArgs& a, const SegArgs& sg, hipStream_t st) {
  PSI_REQUIRE(op->seg_sliced, "sliced layout not built");
  SliceArgs sa{};
  sa.S = sg.S;
  sa.respect_done = a.respect_done;
  sa.x = a.x;
  sa.row = op->slice_row;
  sa.len = op->slice_len;
  sa.col = op->slice_col;
  sa.seg_col = op->seg_col;
  sa.chunk = op->slice_chunk;
  sa.part = op->slice_part;
  sa.ticket = op->slice_ticket;
  sa.ctrl = a.ctrl;
  sa.gap_prev = a.gap_prev;
  sa.hist = a.hist;
  sa.count_iter = a.count_iter;
  sa.defer_gap = a.defer_gap;
  sa.pass_id = a.pass_id;
  int most = 0;
  for (int s = 0; s < sg.S; ++s) {
    sa.seg[s].slices = op->slice_desc + op->seg_slice0[s];
    sa.seg[s].n_slices = op->seg_slice0[s + 1] - op->seg_slice0[s];
    sa.seg[s].y = sg.seg[s].y;
    most = std::max(most, sa.seg[s].n_slices);
  }
  const int per_round = 8 / sg.S;
  const int64_t ranks = (int64_t(most) + kBlock / 64 - 1) / (kBlock / 64);
  const int64_t grid = 8 * std::max<int64_t>(1, (ranks + per_round - 1) / per_round);
  PSI_REQUIRE(grid <= int64_t(1) << 30, "too many slices for one launch");
  hipLaunchKernelGGL(k_slices<MODE>, dim3(unsigned(grid)), dim3(kBlock), 0, st, sa);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

template <int MODE, class YT>
psi_status launch_combine(const PassArgs& a, const SegArgs& sg, hipStream_t st) {
  // about four rows per thread and round; at most 1024 workgroups
  const int want = static_cast<int>((a.n_rows + 4 * kBlock - 1) / (4 * kBlock));
  const int grid = std::max(1, std::min(1024, want));
  hipLaunchKernelGGL((k_combine<MODE, YT>), dim3(grid), dim3(kBlock), 0, st, a, sg);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

template <int MODE, int R, int NW>
psi_status launch_bands_r(psi_operator* op, const PassArgs& a, bool band_only, hipStream_t st) {
  BandArgs b{};
  b.ent = op->band_ent;
  b.toff = op->band_toff;
  b.blocks = op->band_blocks;
  b.piece = op->band_piece;
  b.pairs = op->band_pairs;
  b.B = op->band_B;
  b.wlog = op->band_wlog;
  b.n_blocks = op->band_nb;
  b.pace = op->band_pace_ticks;
  const bool gs = a.gs_sweep && MODE == kStep64;
  b.x_new = gs ? static_cast<const void*>(a.z_new) : nullptr;
  BandFixArgs f{};
  f.split = op->band_split;
  f.piece = op->band_piece;
  f.pairs = op->band_pairs;
  const int wg_per_band = op->band_waves / NW;
  // pairs: the band launches' workgroups first, then one per band for the split
  // rows a Gauss–Seidel sweep finishes after that band
  const int band_pairs = (op->band_nb + NW - 1) / NW;
  int n_pairs = 0;
  for (int k = 0; k < op->band_count; ++k) {
    b.first_block = k * op->band_waves;
    const int nb = std::min(op->band_waves, op->band_nb - b.first_block);
    const int grid = (nb + NW - 1) / NW;
    b.pair_base = k * wg_per_band;
    b.first_launch = k == 0;
    b.fresh_below = gs ? op->band_row0[k] : 0;
    if (gs)
      hipLaunchKernelGGL((k_band<MODE, R, NW, true>), dim3(grid), dim3(NW * 64), 0, st, a, b);
    else
      hipLaunchKernelGGL((k_band<MODE, R, NW, false>), dim3(grid), dim3(NW * 64), 0, st, a, b);
    n_pairs = b.pair_base + grid;
    if (gs) {
      const int lo = k ? op->band_split_end[k - 1] : 0, hi = op->band_split_end[k];
      hipLaunchKernelGGL(k_band_split<MODE>, dim3(1), dim3(kBlock), 0, st, a, f, lo, hi,
                         band_pairs + k, 0);
    }
  }
  PSI_HIP_CHECK(hipGetLastError());
  if (band_only) return PSI_OK;
  f.n_split = gs ? 0 : op->band_n_split;
  f.n_pairs = MODE == kFinal64 ? 0 : (gs ? band_pairs + op->band_count : n_pairs);
  const int want = std::max((f.n_split + kBlock - 1) / kBlock, (f.n_pairs + 255) / 256);
  const int grid = std::max(1, std::min(kBandFixGrid, want));
  hipLaunchKernelGGL(k_band_fix<MODE>, dim3(grid), dim3(kBlock), 0, st, a, f);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

template <int MODE>
psi_status launch_bands_mode(psi_operator* op, const PassArgs& a, bool band_only,
                             hipStream_t st) {
  switch (op->band_rows) {
    case 2048: return launch_bands_r<MODE, 2048, 4>(op, a, band_only, st);
    case 1536: return launch_bands_r<MODE, 1536, 4>(op, a, band_only, st);
    case 1280: return launch_bands_r<MODE, 1280, 4>(op, a, band_only, st);
    default: return launch_bands_r<MODE, 1024, 4>(op, a, band_only, st);
  }
}

// A binned pass: expand, bins, then the split rows and the gap (k_band_fix).
template <int MODE>
psi_status launch_bins_mode(psi_operator* op, const PassArgs& a, hipStream_t st) {
  using XT = typename std::conditional<MODE == kStep32, float, double>::type;
  BinsArgs b{};
  b.col = op->bins_col;
  b.row = op->bins_row;
  b.val = op->bins_val;
  b.rdelta = op->bins_rdelta;
  b.cs = op->bins_cs;
  b.task = op->bins_task;
  b.bstart = op->bins_bstart;
  b.order = op->bins_order;
  b.blocks = op->bins_blocks;
  b.piece = op->bins_piece;
  b.pairs = op->bins_pairs;
  b.B = op->bins_B;
  b.per_xcd = (op->bins_B + 7) / 8;
  b.nb = op->bins_nb;
  b.runs = static_cast<uint32_t>(op->bins_runs);
  b.m = static_cast<uint32_t>(op->m);
  hipLaunchKernelGGL(k_bins_expand<XT>, dim3(unsigned(8 * b.per_xcd)),
                     dim3(kBinsExpandWaves * 64), 0, st, a, b);
  const int grid = (b.nb + kBinsWaves - 1) / kBinsWaves;
  hipLaunchKernelGGL((k_bins<MODE, kBinsRows, kBinsWaves>), dim3(unsigned(std::max(1, grid))),
                     dim3(kBinsWaves * 64), 0, st, a, b);
  BandFixArgs f{};
  f.split = op->bins_split;
  f.piece = op->bins_piece;
  f.pairs = op->bins_pairs;
  f.n_split = op->bins_n_split;
  f.n_pairs = MODE == kFinal64 ? 0 : grid;
  const int want = std::max((f.n_split + kBlock - 1) / kBlock, (f.n_pairs + 255) / 256);
  const int fgrid = std::max(1, std::min(kBandFixGrid, want));
  hipLaunchKernelGGL(k_band_fix<MODE>, dim3(fgrid), dim3(kBlock), 0, st, a, f);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

// Co-resident workgroups of a kernel of `threads` threads per workgroup.
template <class K>
int resident_groups(K kernel, int threads, int max_per_cu = 1 << 20) {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
    return 0;
  return std::min(max_per_cu, std::max(1, per_cu)) * cus;
}

}  // namespace

int band_waves(int rows) {
  // every workgroup of a launch resident at once, at most four per CU, up to
  // the capacities' cap.  Five 1024-row workgroups fit a CU's LDS, but the
  // launch then runs slower per row at every pacing (40M users: 24.6 ms per
  // pass at best against 18.6 ms with four): more waves in flight spread
  // over more column blocks, and the gathers miss the L2 more often
  int groups = 0;
  switch (rows) {
    case 2048: groups = resident_groups(k_band<kStep64, 2048, 4, false>, 4 * 64, 4); break;
    case 1536: groups = resident_groups(k_band<kStep64, 1536, 4, false>, 4 * 64, 4); break;
    case 1280: groups = resident_groups(k_band<kStep64, 1280, 4, false>, 4 * 64, 4); break;
    default: groups = resident_groups(k_band<kStep64, 1024, 4, false>, 4 * 64, 4); break;
  }
  const int waves = groups * 4;
  return std::min(kBandWaveCap, waves);
}

psi_status launch_pass_bands(psi_operator* op, PassMode mode, const PassArgs& a, bool band_only,
                             hipStream_t st) {
  PSI_REQUIRE(op->band_built, "band layout not built");
  switch (mode) {
    case kStep64: return launch_bands_mode<kStep64>(op, a, band_only, st);
    case kFinal64: return launch_bands_mode<kFinal64>(op, a, band_only, st);
    case kStep32: return launch_bands_mode<kStep32>(op, a, band_only, st);
    default: break;
  }
  set_error("this pass has no band form");
  return PSI_EINVAL;
}

psi_status launch_pass_bins(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t st) {
  PSI_REQUIRE(op->bins_built, "binned layout not built");
  switch (mode) {
    case kStep64: return launch_bins_mode<kStep64>(op, a, st);
    case kFinal64: return launch_bins_mode<kFinal64>(op, a, st);
    case kStep32: return launch_bins_mode<kStep32>(op, a, st);
    default: break;
  }
  set_error("this pass has no binned form");
  return PSI_EINVAL;
}

psi_status run_pass(psi_operator* op, int S, PassMode mode, const PassArgs& a, hipStream_t st) {
  if (op->seg_form == kSegBands && (mode == kStep64 || mode == kFinal64 || mode == kStep32))
    return launch_pass_bands(op, mode, a, false, st);
  if (op->seg_form == kSegBins && (mode == kStep64 || mode == kFinal64 || mode == kStep32))
    return launch_pass_bins(op, mode, a, st);
  if (S > 1 && mode != kStep64W) return launch_pass_seg(op, mode, a, st);
  return launch_pass(op, mode, a, st);
}

psi_status launch_gap_decide(Ctrl* ctrl, double* pairs, double* hist, int count_iter,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_gap_decide, dim3(1), dim3(kBlock), 0, st, ctrl, pairs, hist, count_iter);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

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
  a.graph_of = op->graph_of;
  a.inv_ng = op->inv_ng;
  a.gdone = op->gdone;
  a.row_delta = op->row_delta;
  a.part_open = op->part_open;
  a.gap_part = op->gap_part;
  a.gap_grp = op->gap_grp;
  a.grp_ticket = op->grp_ticket;
  a.ctrl = op->ctrl;
  a.hist = op->hist;
  a.defer_gap = 0;
  a.pass_id = kNoPass;
  return a;
}

psi_status launch_pass(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t st) {
  (void)op;
  switch (mode) {
    case kStep64: return launch_mode<kStep64>(a, st);
    case kStep64W: return launch_mode<kStep64W>(a, st);
    case kFinal64: return launch_mode<kFinal64>(a, st);
    case kStep32: return launch_mode<kStep32>(a, st);
    case kStep64G: return launch_mode<kStep64G>(a, st);
    case kFinal64G: return launch_mode<kFinal64G>(a, st);
    case kStep32G: return launch_mode<kStep32G>(a, st);
    default: break;
  }
  set_error("unknown pass mode");
  return PSI_EINVAL;
}

// The partial kernel of a segmented pass in the operator's current form.
template <int PMODE>
psi_status launch_partial(psi_operator* op, const PassArgs& a, const SegArgs& sg, hipStream_t st) {
  if (op->seg_form == kSegSlices) return launch_slices<PMODE>(op, a, sg, st);
  PSI_REQUIRE(op->seg_form == kSegTiles && op->seg_items > 0, "segment layout not prepared");
  PassArgs b = a;
  b.tile_items = op->seg_items;
  return launch_seg_mode<PMODE>(b, sg, st);
}

// A pass in column-segmented form: partial pass + combine (S = op->seg_S).
psi_status launch_pass_seg(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t st) {
  SegArgs sg{};
  sg.S = op->seg_S;
  for (int s = 0; s < sg.S; ++s) sg.seg[s] = op->seg[s];
  psi_status r = PSI_OK;
  switch (mode) {
    case kStep64:
    case kFinal64:
      for (int s = 0; s < sg.S; ++s) sg.seg[s].y = op->seg_y + size_t(s) * op->n;
      r = launch_partial<kPart64>(op, a, sg, st);
      if (r != PSI_OK) return r;
      return mode == kStep64 ? launch_combine<kStep64, double>(a, sg, st)
                             : launch_combine<kFinal64, double>(a, sg, st);
    case kStep64G:
    case kFinal64G:
      for (int s = 0; s < sg.S; ++s) sg.seg[s].y = op->seg_y + size_t(s) * op->n;
      r = launch_partial<kPart64>(op, a, sg, st);
      if (r != PSI_OK) return r;
      return mode == kStep64G ? launch_combine<kStep64G, double>(a, sg, st)
                              : launch_combine<kFinal64G, double>(a, sg, st);
    case kStep32:
    case kStep32G:
      for (int s = 0; s < sg.S; ++s)
        sg.seg[s].y = reinterpret_cast<float*>(op->seg_y) + size_t(s) * op->n;
      r = launch_partial<kPart32>(op, a, sg, st);
      if (r != PSI_OK) return r;
      return mode == kStep32 ? launch_combine<kStep32, float>(a, sg, st)
                             : launch_combine<kStep32G, float>(a, sg, st);
    default: break;
  }
  set_error("this pass has no column-segmented form");
  return PSI_EINVAL;
}

psi_status launch_part_seg(psi_operator* op, PassMode mode, const PassArgs& a, hipStream_t st) {
  SegArgs sg{};
  sg.S = op->seg_S;
  for (int s = 0; s < sg.S; ++s) sg.seg[s] = op->seg[s];
  if (mode == kStep32) {
    for (int s = 0; s < sg.S; ++s)
      sg.seg[s].y = reinterpret_cast<float*>(op->seg_y) + size_t(s) * op->n;
    return launch_partial<kPart32>(op, a, sg, st);
  }
  for (int s = 0; s < sg.S; ++s) sg.seg[s].y = op->seg_y + size_t(s) * op->n;
  return launch_partial<kPart64>(op, a, sg, st);
}

}  // namespace psi
