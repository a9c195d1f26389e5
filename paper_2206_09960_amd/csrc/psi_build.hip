// Operator build on the device (Sec. II: the definitions of A, b_i, C, d_i).
//
// edges -> drop self-loops -> LSD radix sort of (follower, leader) keys ->
// drop repeats -> CSR(A) (rows = followers j, cols = leaders L(j)) ->
// den_j, 1/den_j, row sums of A and B -> sort of the swapped keys ->
// CSR(Aᵀ) (rows = leaders i, cols = followers j, ascending), the pull
// operator the Power-ψ pass runs over.
//
// Every step is deterministic: the sort is total on (row, col) keys, sums run
// in ascending column order, and maxima are exact.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "psi_internal.h"

namespace psi {

bool tile_items_supported(int t);

namespace {

constexpr int kSortWaves = 4;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortWaves * kSortRounds * 64;  // keys per workgroup
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

inline int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

// ------------------------------------------------------------------ scan
// Exclusive prefix sum of uint32 (results fit in uint32: callers bound the
// totals by 2^31).  Three kernels: tile totals, scan of the totals, tile scan.
__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(const uint32_t* in, int64_t n,
                                                           uint32_t* tile_sums) {
  __shared__ uint32_t red[kBlock / 64];
  int64_t base = int64_t(blockIdx.x) * kScanTile;
  uint32_t acc = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t k = base + int64_t(i) * kBlock + threadIdx.x;
    if (k < n) acc += in[k];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    tile_sums[blockIdx.x] = t;
  }
}

// Single workgroup: exclusive scan of the tile totals, chunk by chunk.
__global__ __launch_bounds__(1024) void k_scan_totals(uint32_t* sums, int64_t n_tiles,
                                                      uint32_t* total_out) {
  __shared__ uint32_t buf[1024];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n_tiles; base += 1024) {
    int64_t k = base + threadIdx.x;
    uint32_t v = k < n_tiles ? sums[k] : 0u;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      uint32_t t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0u;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    uint32_t incl = buf[threadIdx.x];
    if (k < n_tiles) sums[k] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += incl;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t* in, uint32_t* out,
                                                       int64_t n, const uint32_t* tile_off) {
  __shared__ uint32_t part[kBlock];
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint32_t run = 0;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t k = base + i;
    v[i] = k < n ? in[k] : 0u;
    run += v[i];
  }
  part[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    uint32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t acc = tile_off[blockIdx.x] + part[threadIdx.x] - run;
  for (int i = 0; i < kScanItems; ++i) {
    int64_t k = base + i;
    if (k < n) out[k] = acc;
    acc += v[i];
  }
}

// ------------------------------------------------------------------ radix sort
// LSD radix sort of uint64 keys, 8-bit digits.  A workgroup owns kSortTile
// consecutive keys; wave w takes rounds of 64 consecutive keys, so the order
// (wave, round, lane) is the input order and the scatter is stable.
__device__ inline uint64_t lanemask_lt() {
  return (uint64_t(1) << __lane_id()) - 1;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* keys, int64_t n, int shift,
                                                       uint32_t* counts, int n_blocks) {
  __shared__ uint32_t hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = int64_t(blockIdx.x) * kSortTile;
  for (int i = 0; i < kSortTile / kBlock; ++i) {
    int64_t k = base + int64_t(i) * kBlock + threadIdx.x;
    if (k < n) atomicAdd(&hist[(keys[k] >> shift) & 255u], 1u);
  }
  __syncthreads();
  counts[int64_t(threadIdx.x) * n_blocks + blockIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t* keys_in,
                                                          uint64_t* keys_out, int64_t n,
                                                          int shift, const uint32_t* offsets,
                                                          int n_blocks) {
  __shared__ uint32_t wave_cnt[kSortWaves][256];
  __shared__ uint32_t glob[256];
  __shared__ uint32_t loff[256];         // first slot of each digit in the staged tile
  __shared__ uint32_t wsum[kSortWaves];
  __shared__ uint64_t stage[kSortTile];  // the tile's keys, stably grouped by digit
  const int wave = threadIdx.x >> 6;
  const int lane = __lane_id();
  for (int w = 0; w < kSortWaves; ++w) wave_cnt[w][threadIdx.x] = 0;
  glob[threadIdx.x] = offsets[int64_t(threadIdx.x) * n_blocks + blockIdx.x];
  __syncthreads();
  const int64_t tile0 = int64_t(blockIdx.x) * kSortTile;
  int64_t base = tile0 + int64_t(wave) * (kSortRounds * 64);
  uint64_t key[kSortRounds];
  uint32_t pos[kSortRounds];
  for (int r = 0; r < kSortRounds; ++r) {
    int64_t k = base + int64_t(r) * 64 + lane;
    bool valid = k < n;
    key[r] = valid ? keys_in[k] : 0;
    uint32_t dig = uint32_t(key[r] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      bool bit = (dig >> b) & 1u;
      uint64_t m = __ballot(valid && bit);
      peers &= bit ? m : ~m;
    }
    uint32_t rank = __popcll(peers & lanemask_lt());
    uint32_t before = wave_cnt[wave][dig];
    pos[r] = before + rank;
    if (valid && rank == 0) wave_cnt[wave][dig] = before + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // digit t (thread t): the waves' exclusive prefix in wave order, the total
  uint32_t total = 0;
  for (int w = 0; w < kSortWaves; ++w) {
    const uint32_t t = wave_cnt[w][threadIdx.x];
    wave_cnt[w][threadIdx.x] = total;
    total += t;
  }
  // exclusive scan of the 256 digit totals: the digit's first slot in the tile
  uint32_t incl = total;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  loff[threadIdx.x] = before + incl - total;
  __syncthreads();
  // stage every key at its place in the tile's stable digit order ...
  for (int r = 0; r < kSortRounds; ++r) {
    int64_t k = base + int64_t(r) * 64 + lane;
    if (k < n) {
      uint32_t dig = uint32_t(key[r] >> shift) & 255u;
      stage[loff[dig] + wave_cnt[wave][dig] + pos[r]] = key[r];
    }
  }
  __syncthreads();
  // ... and write each digit's run out, consecutive threads on consecutive
  // addresses (the same positions as writing every key from its own lane)
  const int cnt = static_cast<int>(n - tile0 < kSortTile ? n - tile0 : kSortTile);
  for (int i = threadIdx.x; i < cnt; i += kBlock) {
    const uint64_t v = stage[i];
    const uint32_t dig = uint32_t(v >> shift) & 255u;
    const uint64_t p = uint64_t(glob[dig]) + uint32_t(i - loff[dig]);
    if (p < uint64_t(n)) keys_out[p] = v;
  }
}

// ------------------------------------------------------------------ edge kernels
__global__ void k_check_activity(const double* lam, const double* mu, int64_t n, Ctrl* ctrl) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double l = lam[i], m = mu[i];
  if (!(l > 0.0) || !isfinite(l) || !(m >= 0.0) || !isfinite(m))
    atomicOr(&ctrl->err_flags, kErrActivity);
}

// key = (row << nb) | col; self-loops become the all-ones sentinel, which
// sorts after every real key and is dropped by the compaction.
__global__ void k_pack_keys(const int32_t* follower, const int32_t* leader, int64_t m,
                            int64_t n, int nb, int follower_major, uint64_t sentinel,
                            const int64_t* graph_off, int n_graphs, uint64_t* keys,
                            Ctrl* ctrl) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  int64_t f = follower[k], l = leader[k];
  if (f < 0 || f >= n || l < 0 || l >= n) {
    atomicOr(&ctrl->err_flags, kErrIndex);
    keys[k] = sentinel;
    return;
  }
  if (n_graphs > 1) {
    // graph of a user: last g with graph_off[g] <= id
    int lo = 0, hi = n_graphs;
    while (hi - lo > 1) {
      int mid = lo + ((hi - lo) >> 1);
      if (graph_off[mid] <= f) lo = mid; else hi = mid;
    }
    if (l < graph_off[lo] || l >= graph_off[lo + 1]) atomicOr(&ctrl->err_flags, kErrCrossGraph);
  }
  if (f == l) {
    atomicAdd(&ctrl->n_self_loops, 1ull);
    keys[k] = sentinel;
    return;
  }
  uint64_t row = uint64_t(follower_major ? f : l);
  uint64_t cl = uint64_t(follower_major ? l : f);
  keys[k] = (row << nb) | cl;
}

__global__ void k_flag_unique(const uint64_t* keys, int64_t m, uint64_t sentinel,
                              uint32_t* flags) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  uint64_t v = keys[k];
  flags[k] = (v != sentinel && (k == 0 || keys[k - 1] != v)) ? 1u : 0u;
}

__global__ void k_compact(const uint64_t* keys, int64_t m, uint64_t sentinel,
                          const uint32_t* pos, uint64_t* out) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  uint64_t v = keys[k];
  if (v != sentinel && (k == 0 || keys[k - 1] != v)) out[pos[k]] = v;
}

__global__ void k_swap_halves(const uint64_t* in, int64_t m, int nb, uint64_t* out) {
  int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= m) return;
  uint64_t v = in[k];
  uint64_t mask = (uint64_t(1) << nb) - 1;
  out[k] = ((v & mask) << nb) | (v >> nb);
}

// CSR from row-major sorted distinct keys: col[e] and the row starts.
__global__ void k_csr_from_keys(const uint64_t* keys, int64_t m, int64_t n, int nb,
                                int* row_ptr, int* col) {
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  uint64_t v = keys[e];
  uint64_t mask = (uint64_t(1) << nb) - 1;
  int64_t r = int64_t(v >> nb);
  col[e] = int(v & mask);
  int64_t r_prev = e == 0 ? -1 : int64_t(keys[e - 1] >> nb);
  for (int64_t rr = r_prev + 1; rr <= r; ++rr) row_ptr[rr] = int(e);
  if (e == m - 1)
    for (int64_t rr = r + 1; rr <= n; ++rr) row_ptr[rr] = int(m);
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_int(int* p, int64_t n, int v) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Per follower j over CSR(A): den_j = Σ_{ℓ∈L(j)}(λ_ℓ+μ_ℓ) in ascending ℓ,
// 1/den_j (0 for an empty newsfeed), and the row sums of B and A.
// Maxima of non-negative doubles (bit patterns order like the values) and a
// count, reduced over the workgroup and added with one atomic each: the
// control block takes one atomic per workgroup, never one per user.
__device__ inline void block_max2_count(double bm, double km, unsigned long long cnt,
                                        unsigned long long* bm_bits, unsigned long long* km_bits,
                                        unsigned long long* count) {
  __shared__ double rb[kBlock / 64], rk[kBlock / 64];
  __shared__ unsigned long long rc[kBlock / 64];
  for (int off = 32; off > 0; off >>= 1) {
    bm = fmax(bm, __shfl_xor(bm, off, 64));
    km = fmax(km, __shfl_xor(km, off, 64));
    cnt += __shfl_xor(cnt, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rb[w] = bm;
    rk[w] = km;
    rc[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kBlock / 64; ++i) {
      bm = fmax(bm, rb[i]);
      km = fmax(km, rk[i]);
      cnt += rc[i];
    }
    if (bm_bits) atomicMax(bm_bits, (unsigned long long)__double_as_longlong(bm));
    if (km_bits) atomicMax(km_bits, (unsigned long long)__double_as_longlong(km));
    if (count && cnt) atomicAdd(count, cnt);
  }
}

// Per follower j over CSR(A): den_j = Σ_{ℓ∈L(j)}(λ_ℓ+μ_ℓ) in ascending ℓ,
// 1/den_j (0 for an empty newsfeed), and the row sums of B and A.  The grid
// strides over the followers.
// (λ_i, μ_i) side by side, so den reads one 16-byte record per leader.
__global__ void k_pack_rates(const double* lam, const double* mu, int64_t n, double2* rates) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) rates[i] = make_double2(lam[i], mu[i]);
}

__global__ __launch_bounds__(kBlock) void k_den(const int* fm_row_ptr, const int* fm_col,
                                                const double2* rates, int64_t n,
                                                double* invden, Ctrl* ctrl) {
  double bmax = 0.0, kmax = 0.0;  // row sums of B and A
  unsigned long long n_empty = 0;
  for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
       j += int64_t(gridDim.x) * blockDim.x) {
    const int e0 = fm_row_ptr[j], e1 = fm_row_ptr[j + 1];
    double den = 0.0, sl = 0.0, sm = 0.0;
    int e = e0;
    for (; e + 4 <= e1; e += 4) {  // four leaders' rates in flight, added in order
      int k[4];
      double lk[4], mk[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) k[u] = fm_col[e + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 r = rates[k[u]];
        lk[u] = r.x;
        mk[u] = r.y;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        den += lk[u] + mk[u];
        sl += lk[u];
        sm += mk[u];
      }
    }
    for (; e < e1; ++e) {
      const double2 r = rates[fm_col[e]];
      const double lk = r.x, mk = r.y;
      den += lk + mk;
      sl += lk;
      sm += mk;
    }
    if (e1 == e0) {
      invden[j] = 0.0;
      ++n_empty;
    } else {
      const double inv = 1.0 / den;
      invden[j] = inv;
      bmax = fmax(bmax, sl * inv);
      kmax = fmax(kmax, sm * inv);
    }
  }
  block_max2_count(bmax, kmax, n_empty, &ctrl->bnorm_bits, &ctrl->kappa_bits,
                   &ctrl->n_no_leaders);
}

__global__ void k_node_consts(const double* lam, const double* mu, const double* invden,
                              int64_t n, double* c, double* d, float* mu32, float* invden32,
                              float* c32) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double l = lam[i], m = mu[i];
  double ci = m / (l + m);
  c[i] = ci;
  d[i] = l / (l + m);
  mu32[i] = float(m);
  invden32[i] = float(invden[i]);
  c32[i] = float(ci);
}

// Graph of every user and 1/N of that graph (block-diagonal operators).
__global__ void k_graph_rows(const int64_t* graph_off, int n_graphs, int64_t n, int* graph_of,
                             double* inv_ng) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int lo = 0, hi = n_graphs;
  while (hi - lo > 1) {
    int mid = lo + ((hi - lo) >> 1);
    if (graph_off[mid] <= i) lo = mid; else hi = mid;
  }
  graph_of[i] = lo;
  inv_ng[i] = 1.0 / static_cast<double>(graph_off[lo + 1] - graph_off[lo]);
}

// Longest row; the grid strides over the rows and each workgroup adds its
// maximum with one atomic.
__global__ __launch_bounds__(kBlock) void k_max_row(const int* row_ptr, int64_t n, Ctrl* ctrl) {
  __shared__ unsigned long long red[kBlock / 64];
  unsigned long long len = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    len = max(len, (unsigned long long)(row_ptr[i + 1] - row_ptr[i]));
  for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = len;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) len = max(len, red[w]);
    if (len) atomicMax(&ctrl->max_row, len);
  }
}

// a_ji = μ_i / den_j stored per edge of CSR(Aᵀ) row i (weighted form), one
// thread per edge, the row and column read from the edge's sorted key.
__global__ void k_weights64(const uint64_t* keys, int64_t m, int nb, const double* mu,
                            const double* invden, double* val) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint64_t v = keys[e];
  const uint64_t mask = (uint64_t(1) << nb) - 1;
  val[e] = mu[int64_t(v >> nb)] * invden[int64_t(v & mask)];
}

// First row of every merge-path tile: on the path that merges the row ends
// row_ptr[1..n] with the edge indices 0..m-1, tile b starts at diagonal b*T.
__global__ void k_schedule(const int* row_ptr, int64_t n, int64_t m, int64_t items,
                           int64_t n_tiles, int* tile_row) {
  int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b > n_tiles) return;
  int64_t diag = std::min(b * items, n + m);
  int64_t lo = std::max<int64_t>(diag - m, 0), hi = std::min<int64_t>(diag, n);
  while (lo < hi) {
    int64_t pivot = (lo + hi) >> 1;
    if (int64_t(row_ptr[pivot + 1]) <= diag - pivot - 1) lo = pivot + 1; else hi = pivot;
  }
  tile_row[b] = int(lo);
}

// Entries of row i of CSR(Aᵀ) that fall in column segment s (columns are
// ascending within a row, so each segment is a contiguous run): counts.
__global__ void k_seg_count(const int* row_ptr, const int* col, int64_t n, int S, int64_t seg,
                            int* seg_row_ptr) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int lo_e = row_ptr[i];
  const int end = row_ptr[i + 1];
  for (int s = 0; s < S; ++s) {
    // first entry with col >= (s+1)*seg
    const int64_t bound = (s + 1) * seg;
    int lo = lo_e, hi = end;
    while (lo < hi) {
      const int mid = lo + ((hi - lo) >> 1);  // lo + hi can exceed 2^31 past edge 2^30
      if (col[mid] < bound) lo = mid + 1; else hi = mid;
    }
    seg_row_ptr[int64_t(s) * (n + 1) + i] = lo - lo_e;
    lo_e = lo;
  }
}

// Copy each row's run of segment s into that segment's CSR, edge-parallel
// (a hub row is spread over many threads): thread t moves edges
// kSegScatterEdges·t onwards, finds its first edge's row by binary search
// over the row ends and steps to later rows as it goes.  A row's columns
// ascend, so its entries of segment s are one run, which starts after the
// row's entries of the segments before s.
constexpr int kSegScatterEdges = 8;
__global__ void k_seg_scatter(const int* row_ptr, const int* col, int64_t n, int64_t m, int S,
                              int64_t seg, const int* seg_row_ptr, const int64_t* seg_off,
                              int* seg_col) {
  const int64_t e_lo = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) * kSegScatterEdges;
  if (e_lo >= m) return;
  const int64_t e_hi = e_lo + kSegScatterEdges < m ? e_lo + kSegScatterEdges : m;
  // the first row whose end exceeds e_lo holds edge e_lo (row_ptr[n] = m > e_lo)
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (row_ptr[mid + 1] > e_lo) hi = mid; else lo = mid + 1;
  }
  int64_t row = lo;
  int64_t r_end = row_ptr[row + 1];
  int cnt[8];  // the row's entries in each segment
  auto load_counts = [&]() {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int* rp = seg_row_ptr + int64_t(s) * (n + 1);
      cnt[s] = s < S ? rp[row + 1] - rp[row] : 0;
    }
  };
  load_counts();
  for (int64_t e = e_lo; e < e_hi; ++e) {
    while (e >= r_end) {
      ++row;
      r_end = row_ptr[row + 1];
      load_counts();
    }
    const int j = col[e];
    const int s = static_cast<int>(j / seg);
    int64_t run = row_ptr[row];  // start of the row's run of segment s
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2)
      if (s2 < s) run += cnt[s2];
    seg_col[seg_off[s] + seg_row_ptr[int64_t(s) * (n + 1) + row] + (e - run)] = j;
  }
}

// ---------------------------------------------------------------- sliced layout
// One workgroup per window of kSliceWindow rows of one segment; each thread
// owns kSliceWindow / kBlock consecutive rows.
constexpr int kSliceRowsPerThread = kSliceWindow / kBlock;
static_assert(kSliceWindow % kBlock == 0, "window rows must split evenly over the threads");

struct SliceLds {
  int cnt[kSliceShort + 1][kBlock];  // per thread, rows of each length; then their ranks
  int total[kSliceShort + 1];
  int base[kSliceShort + 1];         // first rank of each length (longest first)
  int steps[kSliceWindow / 64];      // steps of each short slice
  int64_t soff[kSliceWindow / 64 + 1];
  int chunk0[kBlock];                // per thread, first chunk / slot of its long rows
  int slot0[kBlock];
  int n_short, n_short_slices, n_chunks, n_slots;
};

struct SegOffsets {
  int64_t off[8];  // first edge of each segment in seg_col
};

// Counts of one window: short rows by length, chunks and slots of long rows;
// thread 0 then derives the short slices and their interleaved entries.
__device__ void plan_window(const int* rp, int64_t w0, int64_t w1, SliceLds& L) {
  const int t = threadIdx.x;
  for (int b = 0; b <= kSliceShort; ++b) L.cnt[b][t] = 0;
  const int64_t r0 = w0 + int64_t(t) * kSliceRowsPerThread;
  const int64_t r1 = r0 + kSliceRowsPerThread < w1 ? r0 + kSliceRowsPerThread : w1;
  int chunks = 0, slots = 0;
  for (int64_t r = r0; r < r1; ++r) {
    const int len = rp[r + 1] - rp[r];
    if (len <= kSliceShort) {
      L.cnt[len][t] += 1;
    } else {
      const int c = (len + kSliceChunk - 1) / kSliceChunk;
      chunks += c;
      if (c > 1) slots += c;
    }
  }
  L.chunk0[t] = chunks;
  L.slot0[t] = slots;
  __syncthreads();
  // exclusive scan over threads of each length's counts (thread b: length b)
  if (t <= kSliceShort) {
    int acc = 0;
    for (int u = 0; u < kBlock; ++u) {
      const int v = L.cnt[t][u];
      L.cnt[t][u] = acc;
      acc += v;
    }
    L.total[t] = acc;
  }
  if (t == kBlock - 1) {
    int ac = 0, as = 0;
    for (int u = 0; u < kBlock; ++u) {
      const int c = L.chunk0[u], sl = L.slot0[u];
      L.chunk0[u] = ac;
      L.slot0[u] = as;
      ac += c;
      as += sl;
    }
    L.n_chunks = ac;
    L.n_slots = as;
  }
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int b = kSliceShort; b >= 0; --b) {
      L.base[b] = acc;
      acc += L.total[b];
    }
    L.n_short = acc;
    const int ns = (acc + 63) / 64;
    L.n_short_slices = ns;
    // a slice's steps are the length of its first (longest) row, rank 64·j
    int j = 0, cum = 0;
    for (int b = kSliceShort; b >= 0 && j < ns; --b) {
      while (j < ns && 64 * j < cum + L.total[b]) L.steps[j++] = b;
      cum += L.total[b];
    }
    int64_t o = 0;
    for (j = 0; j < ns; ++j) {
      L.soff[j] = o;
      o += 64 * int64_t(L.steps[j]);
    }
    L.soff[ns] = o;
  }
  __syncthreads();
}

// plan[k * stride + window] for k = 0 slices, 1 short slices, 2 interleaved
// entries, 3 chunks, 4 slots (entry `windows` of each row is set to 0 for the
// exclusive scan that follows).
__global__ __launch_bounds__(kBlock) void k_slice_plan(const int* seg_row_ptr, int64_t n,
                                                       int64_t nw, int64_t windows,
                                                       uint32_t* plan) {
  __shared__ SliceLds L;
  const int64_t b = blockIdx.x;
  const int64_t s = b / nw, w = b % nw;
  const int* rp = seg_row_ptr + s * (n + 1);
  const int64_t w0 = w * kSliceWindow;
  const int64_t w1 = w0 + kSliceWindow < n ? w0 + kSliceWindow : n;
  plan_window(rp, w0, w1, L);
  if (threadIdx.x == 0) {
    const int64_t stride = windows + 1;
    plan[0 * stride + b] = uint32_t(L.n_short_slices + L.n_chunks);
    plan[1 * stride + b] = uint32_t(L.n_short_slices);
    plan[2 * stride + b] = uint32_t(L.soff[L.n_short_slices]);
    plan[3 * stride + b] = uint32_t(L.n_chunks);
    plan[4 * stride + b] = uint32_t(L.n_slots);
    if (b == 0)
      for (int k = 0; k < 5; ++k) plan[k * stride + windows] = 0;
  }
}

// Writes the window's slices from the scanned plan: short slices first (rows
// ranked by length, longest first, ties by row), then the chunks of its long
// rows in row order.
__global__ __launch_bounds__(kBlock) void k_slice_fill(const int* seg_row_ptr, const int* seg_col,
                                                       SegOffsets so, int64_t n, int64_t nw,
                                                       int64_t windows, const uint32_t* plan,
                                                       SliceDesc* desc, int* lane_row,
                                                       unsigned char* lane_len, int* scol,
                                                       int4* chunk) {
  __shared__ SliceLds L;
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t s = b / nw, w = b % nw;
  const int* rp = seg_row_ptr + s * (n + 1);
  const int64_t w0 = w * kSliceWindow;
  const int64_t w1 = w0 + kSliceWindow < n ? w0 + kSliceWindow : n;
  plan_window(rp, w0, w1, L);
  const int64_t stride = windows + 1;
  const int64_t q0 = plan[0 * stride + b];              // first slice of the window
  const int64_t lane0 = 64 * int64_t(plan[1 * stride + b]);  // first lane slot
  const int64_t e0 = plan[2 * stride + b];              // first interleaved entry
  const int64_t c0 = plan[3 * stride + b];              // first chunk
  const int64_t p0 = plan[4 * stride + b];              // first slot
  const int ns = L.n_short_slices;
  for (int j = t; j < ns; j += kBlock) {
    SliceDesc d;
    d.off = e0 + L.soff[j];
    d.len = L.steps[j];
    d.tag = int(lane0 + 64 * int64_t(j));
    desc[q0 + j] = d;
  }
  const int* col = seg_col + so.off[s];
  const int64_t r0 = w0 + int64_t(t) * kSliceRowsPerThread;
  const int64_t r1 = r0 + kSliceRowsPerThread < w1 ? r0 + kSliceRowsPerThread : w1;
  int ch = L.chunk0[t], sl = L.slot0[t];
  for (int64_t r = r0; r < r1; ++r) {
    const int beg = rp[r], len = rp[r + 1] - beg;
    if (len <= kSliceShort) {
      const int rank = L.base[len] + L.cnt[len][t]++;
      const int j = rank >> 6, lane = rank & 63;
      lane_row[lane0 + rank] = int(r);
      lane_len[lane0 + rank] = static_cast<unsigned char>(len);
      int* dst = scol + e0 + L.soff[j] + lane;
      for (int k = 0; k < L.steps[j]; ++k) dst[int64_t(k) * 64] = k < len ? col[beg + k] : 0;
    } else {
      const int nc = (len + kSliceChunk - 1) / kSliceChunk;
      const int first = nc > 1 ? int(p0 + sl) : -1;
      for (int i = 0; i < nc; ++i) {
        SliceDesc d;
        d.off = so.off[s] + beg + int64_t(i) * kSliceChunk;
        d.len = len - i * kSliceChunk < kSliceChunk ? len - i * kSliceChunk : kSliceChunk;
        d.tag = -1 - int(c0 + ch);
        desc[q0 + ns + ch] = d;
        chunk[c0 + ch] = make_int4(int(r), nc > 1 ? first + i : -1, first, nc);
        ++ch;
      }
      if (nc > 1) sl += nc;
    }
  }
  // lane slots past the last short row: no row, padding entries
  for (int rank = L.n_short + t; rank < 64 * ns; rank += kBlock) {
    const int j = rank >> 6, lane = rank & 63;
    lane_row[lane0 + rank] = -1;
    lane_len[lane0 + rank] = 0;
    int* dst = scol + e0 + L.soff[j] + lane;
    for (int k = 0; k < L.steps[j]; ++k) dst[int64_t(k) * 64] = 0;
  }
}

inline unsigned grid_for(int64_t n, int block = kBlock) {
  return unsigned((n + block - 1) / block);
}

struct Scratch {
  char* p;
  size_t left;
  template <class T>
  T* take(int64_t count) {
    size_t bytes = align_up(size_t(std::max<int64_t>(count, 1)) * sizeof(T));
    if (bytes > left) return nullptr;
    T* r = reinterpret_cast<T*>(p);
    p += bytes;
    left -= bytes;
    return r;
  }
};

struct SortBufs {
  uint64_t* a;
  uint64_t* b;
  uint32_t* counts;   // 256 * n_blocks
  uint32_t* flags;    // m_raw
  uint32_t* tile_sums;
  uint32_t* total;    // 1 value
};

psi_status scan_u32(const uint32_t* in, uint32_t* out, int64_t n, SortBufs& sb,
                    hipStream_t st) {
  if (n <= 0) return PSI_OK;
  int64_t tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(unsigned(tiles)), dim3(kBlock), 0, st, in, n,
                     sb.tile_sums);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, sb.tile_sums, tiles, sb.total);
  hipLaunchKernelGGL(k_scan_apply, dim3(unsigned(tiles)), dim3(kBlock), 0, st, in, out, n,
                     sb.tile_sums);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

// Sorts sb.a[0..m) on the low `bits` bits; returns the buffer holding the result.
// LSD passes over the 8-bit digits from bit first_bit up: a caller whose keys
// are already ordered by their bits below first_bit (within every run of equal
// higher bits) skips those digits.
psi_status radix_sort(SortBufs& sb, int64_t m, int bits, hipStream_t st, uint64_t** result,
                      int first_bit = 0) {
  int n_blocks = int((m + kSortTile - 1) / kSortTile);
  uint64_t* src = sb.a;
  uint64_t* dst = sb.b;
  for (int shift = first_bit; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(n_blocks), dim3(kBlock), 0, st, src, m, shift,
                       sb.counts, n_blocks);
    psi_status s = scan_u32(sb.counts, sb.counts, int64_t(256) * n_blocks, sb, st);
    if (s != PSI_OK) return s;
    hipLaunchKernelGGL(k_radix_scatter, dim3(n_blocks), dim3(kBlock), 0, st, src, dst, m, shift,
                       sb.counts, n_blocks);
    PSI_HIP_CHECK(hipGetLastError());
    std::swap(src, dst);
  }
  *result = src;
  return PSI_OK;
}

}  // namespace

// ------------------------------------------------------------------ layout
static void layout_persistent(int64_t n, int64_t m_raw, int n_graphs, uint32_t flags,
                              psi_operator* op, char* base, size_t* total) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(std::max<size_t>(bytes, 1));
    return p;
  };
  int64_t max_tiles = (n + m_raw) / kMinTileItems + 2;
  char* row_ptr = take(4 * size_t(n + 1));
  char* col = take(4 * size_t(m_raw));
  char* fm_row_ptr = take(4 * size_t(n + 1));
  char* fm_col = take(4 * size_t(m_raw));
  char* graph_of = n_graphs > 1 ? take(4 * size_t(n)) : nullptr;
  char* inv_ng = n_graphs > 1 ? take(8 * size_t(n)) : nullptr;
  char* row_delta = n_graphs > 1 ? take(8 * size_t(n)) : nullptr;
  // per-graph state: the graphs' own iteration, then their correction solves
  char* gdone = n_graphs > 1 ? take(4 * 2 * size_t(n_graphs)) : nullptr;
  char* gskip = n_graphs > 1 ? take(4 * 2 * size_t(n_graphs)) : nullptr;
  char* giter = n_graphs > 1 ? take(4 * 2 * size_t(n_graphs)) : nullptr;
  char* gstatus = n_graphs > 1 ? take(4 * 2 * size_t(n_graphs)) : nullptr;
  char* ggap = n_graphs > 1 ? take(8 * 2 * size_t(n_graphs)) : nullptr;
  char* gtol = n_graphs > 1 ? take(8 * size_t(n_graphs)) : nullptr;
  char* lam = take(8 * size_t(n));
  char* mu = take(8 * size_t(n));
  char* c = take(8 * size_t(n));
  char* d = take(8 * size_t(n));
  char* invden = take(8 * size_t(n));
  char* mu32 = take(4 * size_t(n));
  char* invden32 = take(4 * size_t(n));
  char* c32 = take(4 * size_t(n));
  char* val64 = (flags & PSI_WEIGHTED_FP64) ? take(8 * size_t(m_raw)) : nullptr;
  char* s_a = take(8 * size_t(n));
  char* s_b = take(8 * size_t(n));
  char* z_a = take(8 * size_t(n));
  char* z_b = take(8 * size_t(n));
  char* e_a = take(4 * size_t(n));
  char* e_b = take(4 * size_t(n));
  char* ze_a = take(4 * size_t(n));
  char* ze_b = take(4 * size_t(n));
  char* r32 = take(4 * size_t(n));
  char* part_open = take(8 * size_t(max_tiles));
  char* gap_part = take(2 * 16 * size_t(kMaxGrid));  // two buffers (deferred gaps alternate)
  char* gap_grp = take(16 * size_t(kMaxGrid / 64));
  char* grp_ticket = take(4 * size_t(kMaxGrid / 64));
  char* tile_row = take(4 * size_t(max_tiles + 1));
  char* ctrl = take(2 * sizeof(Ctrl));
  char* hist = take(8 * size_t(kHistLen));
  char* scal = take(8 * 8);
  char* goff = take(8 * size_t(n_graphs + 1));
  // column segments (S <= 8) and their sliced layout
  const bool segs = true;
  const int64_t nw = (n + kSliceWindow - 1) / kSliceWindow;
  // short slices of a window: ceil(rows / 64); interleaved entries: its short
  // rows' edges plus at most 64·kSliceShort of padding (lengths fall from
  // slice to slice); chunks: at most one per long row plus one per kSliceChunk
  // edges, and a long row has more than kSliceShort edges
  const int64_t cap_chunks = segs ? m_raw / (kSliceShort + 1) + m_raw / kSliceChunk + 8 : 0;
  const int64_t cap_slices = segs ? 8 * (n / 64 + nw + 1) + cap_chunks : 0;
  const int64_t cap_lanes = segs ? 8 * (n + 64 * nw) : 0;
  const int64_t cap_entries = segs ? m_raw + 8 * nw * int64_t(kSliceChunk) : 0;
  char* seg_col = take(4 * size_t(segs ? m_raw : 0));
  char* seg_row_ptr = take(4 * size_t(segs ? 8 * (n + 1) : 0));
  const int64_t max_seg_tiles = segs ? (8 * n + m_raw) / kMinTileItems + 16 : 0;
  char* seg_tile_row = take(4 * size_t(max_seg_tiles + 8));
  char* seg_part_open = take(8 * size_t(max_seg_tiles));
  char* seg_y = take(8 * size_t(segs ? 8 * n : 0));
  char* seg_scan_tmp = take(4 * size_t((8 * nw + n + 1) / 4096 + 16));
  char* slice_desc = take(sizeof(SliceDesc) * size_t(cap_slices));
  char* slice_row = take(4 * size_t(cap_lanes));
  char* slice_len = take(size_t(cap_lanes));
  char* slice_col = take(4 * size_t(cap_entries));
  char* slice_chunk = take(16 * size_t(cap_chunks));
  char* slice_part = take(8 * size_t(cap_chunks));
  char* slice_ticket = take(4 * size_t(cap_chunks));
  char* slice_plan = take(4 * size_t(segs ? 5 * (8 * nw + 1) : 0));
  // column-blocked layout (single-graph operators).  Row blocks: at most
  // n/R closed by their row count, 2M/E closed by their edge budget, 2M/E
  // pieces of split rows and one per split row, where the planner keeps
  // M/E <= n/R + waves of a launch (R >= 1024)
  const bool bands = n_graphs == 1;
  const int64_t band_cols =
      bands ? std::max<int64_t>(1, (n + (int64_t(1) << kBandMinLog) - 1) >> kBandMinLog) : 0;
  const int64_t cap_band_blocks = bands ? 6 * ((n + 1023) / 1024) + 5 * int64_t(kBandWaveCap) + 64 : 0;
  const int64_t cap_band_toff = bands ? cap_band_blocks * band_cols + 1 : 0;
  char* band_ent = take(4 * size_t(bands ? m_raw : 0));
  char* band_toff = take(4 * size_t(cap_band_toff));
  char* band_blocks = take(sizeof(BandBlock) * size_t(cap_band_blocks + 1));
  char* band_split = take(16 * size_t(cap_band_blocks));
  char* band_piece = take(8 * size_t(cap_band_blocks));
  // pairs: one per workgroup of the band launches (four row blocks each) and
  // one per band for the split rows a Gauss–Seidel sweep finishes per band
  char* band_pairs = take(16 * size_t(cap_band_blocks / 4 + cap_band_blocks / 256 + 64));
  char* band_scan_tmp = take(4 * size_t((cap_band_toff + 4095) / 4096 + 8));
  // binned layout (single-graph operators): a value, an expand-order column
  // and a bin-order row per edge, and a run table.  Bins are planned with an
  // edge budget of at least 2.5·R·M/N, so there are at most N/R + 5M/E + 1
  // <= 3·ceil(N/1024) + 1 of them (R >= 1024); runs are the non-empty
  // (column block, bin) pairs
  const bool bins = n_graphs == 1;
  const int64_t bins_cols = bins ? std::max<int64_t>(1, (n + kBinsCols - 1) / kBinsCols) : 0;
  const int64_t cap_bins_blocks = bins ? 3 * ((n + 1023) / 1024) + 8 : 0;
  const int64_t cap_bins_runs =
      bins ? std::min<int64_t>(cap_bins_blocks * bins_cols, std::max<int64_t>(m_raw, 1)) : 0;
  // values (8 bytes an edge); 1 MiB more so that the count tables of small
  // operators fit it during the build
  const size_t bins_val_bytes = bins ? 8 * size_t(m_raw) + (size_t(1) << 20) : 0;
  char* bins_val = take(bins_val_bytes);
  char* bins_col = take(2 * size_t(bins ? m_raw : 0));
  char* bins_row = take(2 * size_t(bins ? m_raw : 0));
  char* bins_rdelta = take(4 * size_t(cap_bins_runs));
  char* bins_cs = take(4 * size_t(bins_cols + 1));
  char* bins_crun = take(4 * size_t(bins_cols + 1));
  char* bins_task = take(4 * size_t(bins_cols * kBinsExpandWaves));
  char* bins_bstart = take(4 * size_t(cap_bins_blocks + 1));
  char* bins_order = take(4 * size_t(cap_bins_blocks));
  char* bins_blocks = take(sizeof(BandBlock) * size_t(cap_bins_blocks + 1));
  char* bins_split = take(16 * size_t(cap_bins_blocks));
  char* bins_piece = take(8 * size_t(cap_bins_blocks));
  char* bins_pairs = take(16 * size_t(cap_bins_blocks / kBinsWaves + 1));
  const int64_t mp_max_hubs = m_raw / (kMpHubEdges + 1) + 1;
  const int64_t mp_max_chunks = m_raw / kMpChunkEdges + mp_max_hubs + 1;
  char* mp[2][3];
  for (int o = 0; o < 2; ++o) {
    mp[o][0] = take(4 * size_t(mp_max_hubs));
    mp[o][1] = take(4 * size_t(mp_max_hubs + 1));
    mp[o][2] = take(4 * size_t(mp_max_chunks));
  }
  *total = off;
  if (!op) return;
  op->row_ptr = (int*)row_ptr;
  op->col = (int*)col;
  op->fm_row_ptr = (int*)fm_row_ptr;
  op->fm_col = (int*)fm_col;
  op->graph_of = (int*)graph_of;
  op->inv_ng = (double*)inv_ng;
  op->row_delta = (double*)row_delta;
  op->gdone = (int*)gdone;
  op->gskip = (int*)gskip;
  op->giter = (int*)giter;
  op->gstatus = (int*)gstatus;
  op->ggap = (double*)ggap;
  op->gtol = (double*)gtol;
  op->lam = (double*)lam;
  op->mu = (double*)mu;
  op->c = (double*)c;
  op->d = (double*)d;
  op->invden = (double*)invden;
  op->mu32 = (float*)mu32;
  op->invden32 = (float*)invden32;
  op->c32 = (float*)c32;
  op->val64 = (double*)val64;
  op->s_a = (double*)s_a;
  op->s_b = (double*)s_b;
  op->z_a = (double*)z_a;
  op->z_b = (double*)z_b;
  op->e_a = (float*)e_a;
  op->e_b = (float*)e_b;
  op->ze_a = (float*)ze_a;
  op->ze_b = (float*)ze_b;
  op->r32 = (float*)r32;
  op->part_open = (double*)part_open;
  op->gap_part = (double*)gap_part;
  op->gap_grp = (double*)gap_grp;
  op->grp_ticket = (unsigned*)grp_ticket;
  op->tile_row = (int*)tile_row;
  op->max_tiles = max_tiles;
  op->ctrl = (Ctrl*)ctrl;
  op->hist = (double*)hist;
  op->scal = (double*)scal;
  op->graph_off = (int64_t*)goff;
  op->seg_col = (int*)seg_col;
  op->seg_row_ptr = (int*)seg_row_ptr;
  op->seg_tile_row = (int*)seg_tile_row;
  op->seg_part_open = (double*)seg_part_open;
  op->max_seg_tiles = max_seg_tiles;
  op->seg_y = (double*)seg_y;
  op->seg_scan_tmp = (uint32_t*)seg_scan_tmp;
  op->slice_desc = (SliceDesc*)slice_desc;
  op->slice_row = (int*)slice_row;
  op->slice_len = (unsigned char*)slice_len;
  op->slice_col = (int*)slice_col;
  op->slice_chunk = (int4*)slice_chunk;
  op->slice_part = (double*)slice_part;
  op->slice_ticket = (unsigned*)slice_ticket;
  op->slice_plan = (uint32_t*)slice_plan;
  op->cap_slices = cap_slices;
  op->cap_lanes = cap_lanes;
  op->cap_entries = cap_entries;
  op->cap_chunks = cap_chunks;
  op->band_ent = (uint32_t*)band_ent;
  op->band_toff = (uint32_t*)band_toff;
  op->band_blocks = (BandBlock*)band_blocks;
  op->band_split = (int4*)band_split;
  op->band_piece = (double*)band_piece;
  op->band_pairs = (double*)band_pairs;
  op->band_scan_tmp = (uint32_t*)band_scan_tmp;
  op->cap_band_blocks = cap_band_blocks;
  op->cap_band_toff = cap_band_toff;
  op->cap_band_cols = band_cols;
  op->band_built = false;
  op->bins_val = bins ? static_cast<void*>(bins_val) : nullptr;
  op->bins_col = (uint16_t*)bins_col;
  op->bins_row = (uint16_t*)bins_row;
  op->bins_rdelta = (uint32_t*)bins_rdelta;
  op->bins_cs = (uint32_t*)bins_cs;
  op->bins_crun = (uint32_t*)bins_crun;
  op->bins_task = (int*)bins_task;
  op->bins_bstart = (uint32_t*)bins_bstart;
  op->bins_order = (int*)bins_order;
  op->bins_blocks = (BandBlock*)bins_blocks;
  op->bins_split = (int4*)bins_split;
  op->bins_piece = (double*)bins_piece;
  op->bins_pairs = (double*)bins_pairs;
  op->cap_bins_blocks = cap_bins_blocks;
  op->cap_bins_runs = cap_bins_runs;
  op->cap_bins_cols = bins_cols;
  op->cap_bins_val = bins_val_bytes;
  op->bins_built = false;
  op->mp_max_hubs = mp_max_hubs;
  op->mp_max_chunks = mp_max_chunks;
  for (int o = 0; o < 2; ++o) {
    op->mp_hubs[o].hub_rows = (int*)mp[o][0];
    op->mp_hubs[o].chunk0 = (uint32_t*)mp[o][1];
    op->mp_hubs[o].chunk_hub = (int*)mp[o][2];
    op->mp_hubs[o].n_hubs = -1;
  }
}

static size_t scratch_size(int64_t n, int64_t m_raw) {
  int64_t sort_blocks = (m_raw + kSortTile - 1) / kSortTile;
  int64_t scan_len = std::max<int64_t>(m_raw, 256 * sort_blocks);
  size_t s = 0;
  s += 2 * align_up(8 * size_t(std::max<int64_t>(m_raw, 1)));        // key buffers
  s += align_up(4 * size_t(256 * std::max<int64_t>(sort_blocks, 1))); // digit counts
  s += align_up(4 * size_t(std::max<int64_t>(m_raw, 1)));            // flags / CSR(A) cols
  s += align_up(4 * size_t((scan_len + kScanTile - 1) / kScanTile + 1));
  s += align_up(4 * 4);                                               // scan total
  s += align_up(4 * size_t(n + 1));                                   // CSR(A) rows
  s += align_up(16 * size_t(n));                                      // (λ, μ) interleaved
  return s;
}

Layout compute_layout(int64_t n, int64_t m_raw, int n_graphs, uint32_t flags) {
  Layout L;
  layout_persistent(n, m_raw, n_graphs, flags, nullptr, nullptr, &L.persistent);
  L.scratch = scratch_size(n, m_raw);
  return L;
}

void carve_persistent(psi_operator* op, char* base, int64_t m_raw, int n_graphs) {
  size_t total = 0;
  layout_persistent(op->n, m_raw, n_graphs, op->flags, op, base, &total);
}

// ------------------------------------------------------------------ build
psi_status build_operator(psi_operator* op, const int32_t* follower, const int32_t* leader,
                          const double* lambda, const double* mu, const int64_t* node_offsets,
                          char* scratch, size_t scratch_bytes, hipStream_t st) {
  const int64_t n = op->n;
  const int64_t m_raw = op->m_in;
  const bool host_in = (op->flags & PSI_INPUT_HOST) != 0;
  Scratch sc{scratch, scratch_bytes};
  SortBufs sb{};
  sb.a = sc.take<uint64_t>(m_raw);
  sb.b = sc.take<uint64_t>(m_raw);
  int64_t sort_blocks = (m_raw + kSortTile - 1) / kSortTile;
  sb.counts = sc.take<uint32_t>(256 * std::max<int64_t>(sort_blocks, 1));
  sb.flags = sc.take<uint32_t>(m_raw);
  int64_t scan_len = std::max<int64_t>(m_raw, 256 * sort_blocks);
  sb.tile_sums = sc.take<uint32_t>((scan_len + kScanTile - 1) / kScanTile + 1);
  sb.total = sc.take<uint32_t>(4);
  int* fm_row_ptr_tmp = sc.take<int>(n + 1);
  double2* rates = sc.take<double2>(n);
  if (!sb.a || !sb.b || !sb.counts || !sb.flags || !sb.tile_sums || !sb.total ||
      !fm_row_ptr_tmp || !rates) {
    set_error("scratch workspace too small");
    return PSI_ENOSPACE;
  }

  PSI_HIP_CHECK(hipMemsetAsync(op->ctrl, 0, 2 * sizeof(Ctrl), st));
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(op->max_tiles)), dim3(kBlock), 0, st,
                     reinterpret_cast<uint64_t*>(op->part_open), op->max_tiles, kEmptySlot);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(4 * kMaxGrid)), dim3(kBlock), 0, st,
                     reinterpret_cast<uint64_t*>(op->gap_part), int64_t(4 * kMaxGrid), kEmptySlot);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(2 * kMaxGrid / 64)), dim3(kBlock), 0, st,
                     reinterpret_cast<uint64_t*>(op->gap_grp), int64_t(2 * kMaxGrid / 64),
                     kEmptySlot);
  PSI_HIP_CHECK(hipMemsetAsync(op->grp_ticket, 0, 4 * size_t(kMaxGrid / 64), st));
  if (op->max_seg_tiles > 0)
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(op->max_seg_tiles)), dim3(kBlock), 0, st,
                       reinterpret_cast<uint64_t*>(op->seg_part_open), op->max_seg_tiles,
                       kEmptySlot);
  op->seg_S = 0;
  if (op->n_graphs > 1)
    PSI_HIP_CHECK(hipMemcpyAsync(op->graph_off, node_offsets, 8 * size_t(op->n_graphs + 1),
                                 hipMemcpyHostToDevice, st));
  // activity vectors -> persistent λ, μ
  hipMemcpyKind kind = host_in ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  PSI_HIP_CHECK(hipMemcpyAsync(op->lam, lambda, 8 * size_t(n), kind, st));
  PSI_HIP_CHECK(hipMemcpyAsync(op->mu, mu, 8 * size_t(n), kind, st));
  hipLaunchKernelGGL(k_check_activity, dim3(grid_for(n)), dim3(kBlock), 0, st, op->lam, op->mu,
                     n, op->ctrl);
  // edges (host copies go to the second key buffer, unused until the first scatter)
  const int32_t* f_dev = follower;
  const int32_t* l_dev = leader;
  if (host_in && m_raw > 0) {
    int32_t* tmp = reinterpret_cast<int32_t*>(sb.b);
    PSI_HIP_CHECK(hipMemcpyAsync(tmp, follower, 4 * size_t(m_raw), hipMemcpyHostToDevice, st));
    PSI_HIP_CHECK(hipMemcpyAsync(tmp + m_raw, leader, 4 * size_t(m_raw), hipMemcpyHostToDevice,
                                 st));
    f_dev = tmp;
    l_dev = tmp + m_raw;
  }
  const int nb = bits_for(n);
  const int key_bits = 2 * nb;
  const uint64_t sentinel = key_bits >= 64 ? ~uint64_t(0) : ((uint64_t(1) << key_bits) - 1);

  int64_t m = 0;
  uint64_t* sorted = sb.a;
  if (m_raw > 0) {
    hipLaunchKernelGGL(k_pack_keys, dim3(grid_for(m_raw)), dim3(kBlock), 0, st, f_dev, l_dev,
                       m_raw, n, nb, 1, sentinel, op->graph_off, op->n_graphs, sb.a, op->ctrl);
    PSI_HIP_CHECK(hipGetLastError());
    psi_status s = radix_sort(sb, m_raw, key_bits, st, &sorted);
    if (s != PSI_OK) return s;
    hipLaunchKernelGGL(k_flag_unique, dim3(grid_for(m_raw)), dim3(kBlock), 0, st, sorted, m_raw,
                       sentinel, sb.flags);
    s = scan_u32(sb.flags, sb.flags, m_raw, sb, st);
    if (s != PSI_OK) return s;
    uint32_t total = 0;
    PSI_HIP_CHECK(hipMemcpyAsync(&total, sb.total, 4, hipMemcpyDeviceToHost, st));
    uint64_t* uniq = (sorted == sb.a) ? sb.b : sb.a;
    hipLaunchKernelGGL(k_compact, dim3(grid_for(m_raw)), dim3(kBlock), 0, st, sorted, m_raw,
                       sentinel, sb.flags, uniq);
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    m = int64_t(total);
    sorted = uniq;
  }
  Ctrl hc{};
  PSI_HIP_CHECK(hipMemcpyAsync(&hc, op->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  if (hc.err_flags & kErrIndex) { set_error("edge endpoint outside [0, n_users)"); return PSI_EINVAL; }
  if (hc.err_flags & kErrActivity) {
    set_error("activity must satisfy lambda > 0 and mu >= 0, both finite");
    return PSI_EINVAL;
  }
  if (hc.err_flags & kErrCrossGraph) { set_error("an edge joins two graphs"); return PSI_EINVAL; }
  const int64_t n_loops = int64_t(hc.n_self_loops);
  const int64_t n_dups = m_raw - n_loops - m;
  if ((op->flags & PSI_STRICT) && (n_loops || n_dups)) {
    set_error("PSI_STRICT: input has " + std::to_string(n_loops) + " self-loops and " +
              std::to_string(n_dups) + " repeated edges");
    return PSI_EINVAL;
  }
  op->m = m;

  // CSR(A): rows = followers j, cols = leaders (in the flags region, or persistent)
  int* fm_row_ptr = op->fm_row_ptr;
  int* fm_col = op->fm_col;
  (void)fm_row_ptr_tmp;
  if (m > 0) {
    hipLaunchKernelGGL(k_csr_from_keys, dim3(grid_for(m)), dim3(kBlock), 0, st, sorted, m, n, nb,
                       fm_row_ptr, fm_col);
  } else {
    hipLaunchKernelGGL(k_fill_int, dim3(grid_for(n + 1)), dim3(kBlock), 0, st, fm_row_ptr, n + 1,
                       0);
  }
  // bounded grids: each workgroup adds its maxima to the control block once
  hipLaunchKernelGGL(k_pack_rates, dim3(grid_for(n)), dim3(kBlock), 0, st, op->lam, op->mu, n,
                     rates);
  hipLaunchKernelGGL(k_den, dim3(std::max(1u, std::min(grid_for(n), 1024u))), dim3(kBlock), 0, st,
                     fm_row_ptr, fm_col, rates, n, op->invden, op->ctrl);
  hipLaunchKernelGGL(k_node_consts, dim3(grid_for(n)), dim3(kBlock), 0, st, op->lam, op->mu,
                     op->invden, n, op->c, op->d, op->mu32, op->invden32, op->c32);
  PSI_HIP_CHECK(hipGetLastError());

  // CSR(Aᵀ): sort the swapped keys
  if (m > 0) {
    uint64_t* other = (sorted == sb.a) ? sb.b : sb.a;
    hipLaunchKernelGGL(k_swap_halves, dim3(grid_for(m)), dim3(kBlock), 0, st, sorted, m, nb,
                       other);
    SortBufs sb2 = sb;
    sb2.a = other;
    sb2.b = sorted;
    uint64_t* res = nullptr;
    // the swapped keys (leader, follower) arrive ordered by follower, their
    // low nb bits, so the digits wholly inside the follower field are already
    // in order: within any run of equal higher bits (same leader, same
    // high follower bits) ascending follower means ascending low bits
    psi_status s = radix_sort(sb2, m, key_bits, st, &res, (nb / 8) * 8);
    if (s != PSI_OK) return s;
    hipLaunchKernelGGL(k_csr_from_keys, dim3(grid_for(m)), dim3(kBlock), 0, st, res, m, n, nb,
                       op->row_ptr, op->col);
    if (op->val64)
      hipLaunchKernelGGL(k_weights64, dim3(grid_for(m)), dim3(kBlock), 0, st, res, m, nb, op->mu,
                         op->invden, op->val64);
  } else {
    hipLaunchKernelGGL(k_fill_int, dim3(grid_for(n + 1)), dim3(kBlock), 0, st, op->row_ptr, n + 1,
                       0);
  }
  hipLaunchKernelGGL(k_max_row, dim3(std::max(1u, std::min(grid_for(n), 256u))), dim3(kBlock), 0,
                     st, op->row_ptr, n, op->ctrl);
  if (op->n_graphs > 1)
    hipLaunchKernelGGL(k_graph_rows, dim3(grid_for(n)), dim3(kBlock), 0, st, op->graph_off,
                       op->n_graphs, n, op->graph_of, op->inv_ng);
  PSI_HIP_CHECK(hipGetLastError());
  PSI_HIP_CHECK(hipMemcpyAsync(&hc, op->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));

  double bnorm, kap;
  std::memcpy(&bnorm, &hc.bnorm_bits, 8);
  std::memcpy(&kap, &hc.kappa_bits, 8);
  psi_operator_stats& S = op->stats;
  S.n_users = n;
  S.n_edges_in = m_raw;
  S.n_edges = m;
  S.n_self_loops = n_loops;
  S.n_duplicates = n_dups;
  S.n_no_leaders = int64_t(hc.n_no_leaders);
  S.max_followers = int64_t(hc.max_row);
  S.n_graphs = op->n_graphs;
  S.flags = int32_t(op->flags);
  S.b_norm = bnorm;
  S.kappa = kap;
  op->sched_items = 0;
  return ensure_schedule(op, kDefaultTileItems, st);
}

psi_status ensure_schedule(psi_operator* op, int tile_items, hipStream_t st) {
  if (tile_items <= 0) tile_items = kDefaultTileItems;
  if (!tile_items_supported(tile_items)) {
    set_error("tile_items must be one of 1024, 1536, 2048, 3072, 4096");
    return PSI_EINVAL;
  }
  if (op->sched_items == tile_items) return PSI_OK;
  int64_t total = op->n + op->m;
  int64_t n_tiles = std::max<int64_t>((total + tile_items - 1) / tile_items, 1);
  if (n_tiles + 1 > op->max_tiles + 1) {
    set_error("schedule does not fit the workspace");
    return PSI_ENOSPACE;
  }
  hipLaunchKernelGGL(k_schedule, dim3(grid_for(n_tiles + 1)), dim3(kBlock), 0, st, op->row_ptr,
                     op->n, op->m, int64_t(tile_items), n_tiles, op->tile_row);
  PSI_HIP_CHECK(hipGetLastError());
  op->sched_items = tile_items;
  op->n_tiles = int(n_tiles);
  return PSI_OK;
}

psi_status ensure_segments(psi_operator* op, int S, hipStream_t st) {
  PSI_REQUIRE(S == 2 || S == 4 || S == 8, "col_segments must be 1, 2, 4 or 8");
  if (op->seg_S == S) return PSI_OK;
  const int64_t n = op->n;
  const int64_t seg = (n + S - 1) / S;
  if (op->m > 0) {
    hipLaunchKernelGGL(k_seg_count, dim3(grid_for(n)), dim3(kBlock), 0, st, op->row_ptr, op->col,
                       n, S, seg, op->seg_row_ptr);
  } else {
    hipLaunchKernelGGL(k_fill_int, dim3(grid_for(int64_t(S) * (n + 1))), dim3(kBlock), 0, st,
                       op->seg_row_ptr, int64_t(S) * (n + 1), 0);
  }
  // exclusive scan of each segment's counts (entry n receives the total)
  SortBufs sb{};
  sb.tile_sums = op->seg_scan_tmp;
  sb.total = op->seg_scan_tmp + ((8 * ((n + kSliceWindow - 1) / kSliceWindow) + n + 1) / 4096 + 8);
  std::vector<uint32_t> totals(S);
  for (int s = 0; s < S; ++s) {
    uint32_t* rp = reinterpret_cast<uint32_t*>(op->seg_row_ptr + int64_t(s) * (n + 1));
    PSI_HIP_CHECK(hipMemsetAsync(rp + n, 0, 4, st));
    psi_status r = scan_u32(rp, rp, n + 1, sb, st);
    if (r != PSI_OK) return r;
    PSI_HIP_CHECK(hipMemcpyAsync(&totals[s], rp + n, 4, hipMemcpyDeviceToHost, st));
  }
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  std::vector<int64_t> off(S + 1, 0);
  for (int s = 0; s < S; ++s) off[s + 1] = off[s] + totals[s];
  if (off[S] != op->m) {
    set_error("column segmentation lost edges");
    return PSI_EDEVICE;
  }
  int64_t* doff = reinterpret_cast<int64_t*>(op->scal);  // 8 values of scratch
  PSI_HIP_CHECK(hipMemcpyAsync(doff, off.data(), 8 * size_t(S), hipMemcpyHostToDevice, st));
  if (op->m > 0)
    hipLaunchKernelGGL(k_seg_scatter,
                       dim3(grid_for((op->m + kSegScatterEdges - 1) / kSegScatterEdges)),
                       dim3(kBlock), 0, st, op->row_ptr, op->col, n, op->m, S, seg,
                       op->seg_row_ptr, doff, op->seg_col);
  PSI_HIP_CHECK(hipGetLastError());
  for (int s = 0; s < S; ++s) {
    op->seg[s].row_ptr = op->seg_row_ptr + int64_t(s) * (n + 1);
    op->seg[s].col = op->seg_col + off[s];
    op->seg[s].n_nnz = static_cast<int>(totals[s]);
  }
  for (int s = 0; s <= S; ++s) op->seg_off[s] = off[s];
  op->seg_S = S;
  op->seg_items = 0;
  op->seg_sliced = false;
  return PSI_OK;
}

// Merge-path schedules of the current segments for tiles of tile_items.
psi_status ensure_seg_tiles(psi_operator* op, int tile_items, hipStream_t st) {
  PSI_REQUIRE(op->seg_S > 1, "no column segments built");
  PSI_REQUIRE(tile_items_supported(tile_items), "unsupported tile_items");
  if (op->seg_items == tile_items) return PSI_OK;
  const int64_t n = op->n;
  int64_t tile_off = 0;
  for (int s = 0; s < op->seg_S; ++s) {
    const int64_t total = n + op->seg[s].n_nnz;
    const int64_t nt = std::max<int64_t>((total + tile_items - 1) / tile_items, 1);
    if (tile_off + nt + 1 > op->max_seg_tiles + 8) {
      set_error("segment schedules do not fit the workspace");
      return PSI_ENOSPACE;
    }
    hipLaunchKernelGGL(k_schedule, dim3(grid_for(nt + 1)), dim3(kBlock), 0, st,
                       op->seg[s].row_ptr, n, int64_t(op->seg[s].n_nnz), int64_t(tile_items), nt,
                       op->seg_tile_row + tile_off);
    op->seg[s].tile_row = op->seg_tile_row + tile_off;
    op->seg[s].part_open = op->seg_part_open + (tile_off - s);
    op->seg[s].n_tiles = static_cast<int>(nt);
    tile_off += nt + 1;
  }
  PSI_HIP_CHECK(hipGetLastError());
  op->seg_items = tile_items;
  return PSI_OK;
}

// Sliced layout of the current segments: per-window counts, their exclusive
// scans, then the fill.
psi_status ensure_seg_slices(psi_operator* op, hipStream_t st) {
  PSI_REQUIRE(op->seg_S > 1, "no column segments built");
  PSI_REQUIRE(op->cap_lanes < (int64_t(1) << 31) && op->cap_chunks < (int64_t(1) << 31),
              "too many users for the sliced layout's 32-bit lane and chunk indices");
  if (op->seg_sliced) return PSI_OK;
  const int64_t n = op->n;
  const int S = op->seg_S;
  SortBufs sb{};
  sb.tile_sums = op->seg_scan_tmp;
  sb.total = op->seg_scan_tmp + ((8 * ((n + kSliceWindow - 1) / kSliceWindow) + n + 1) / 4096 + 8);
  SegOffsets so{};
  for (int s = 0; s < S; ++s) so.off[s] = op->seg_off[s];
  const int64_t nw = (n + kSliceWindow - 1) / kSliceWindow;
  const int64_t windows = int64_t(S) * nw;
  uint32_t* plan = op->slice_plan;
  hipLaunchKernelGGL(k_slice_plan, dim3(unsigned(windows)), dim3(kBlock), 0, st, op->seg_row_ptr,
                     n, nw, windows, plan);
  PSI_HIP_CHECK(hipGetLastError());
  for (int k = 0; k < 5; ++k) {
    uint32_t* row = plan + int64_t(k) * (windows + 1);
    psi_status r = scan_u32(row, row, windows + 1, sb, st);
    if (r != PSI_OK) return r;
  }
  // totals, and the first slice of each segment
  std::vector<uint32_t> tot(5), first(S + 1);
  for (int k = 0; k < 5; ++k)
    PSI_HIP_CHECK(hipMemcpyAsync(&tot[k], plan + int64_t(k) * (windows + 1) + windows, 4,
                                 hipMemcpyDeviceToHost, st));
  for (int s = 0; s <= S; ++s)
    PSI_HIP_CHECK(hipMemcpyAsync(&first[s], plan + int64_t(s) * nw, 4, hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  if (int64_t(tot[0]) > op->cap_slices || 64 * int64_t(tot[1]) > op->cap_lanes ||
      int64_t(tot[2]) > op->cap_entries || int64_t(tot[3]) > op->cap_chunks ||
      int64_t(tot[4]) > op->cap_chunks) {
    set_error("sliced layout exceeds its workspace");
    return PSI_ENOSPACE;
  }
  if (tot[4] > 0) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(tot[4])), dim3(kBlock), 0, st,
                       reinterpret_cast<uint64_t*>(op->slice_part), int64_t(tot[4]), kEmptySlot);
    hipLaunchKernelGGL(k_fill_int, dim3(grid_for(tot[4])), dim3(kBlock), 0, st,
                       reinterpret_cast<int*>(op->slice_ticket), int64_t(tot[4]), 0);
  }
  hipLaunchKernelGGL(k_slice_fill, dim3(unsigned(windows)), dim3(kBlock), 0, st, op->seg_row_ptr,
                     op->seg_col, so, n, nw, windows, plan, op->slice_desc, op->slice_row,
                     op->slice_len, op->slice_col, op->slice_chunk);
  PSI_HIP_CHECK(hipGetLastError());
  for (int s = 0; s <= S; ++s) op->seg_slice0[s] = int(first[s]);
  op->seg_sliced = true;
  return PSI_OK;
}

psi_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tile_sums,
                              uint32_t* total, hipStream_t st) {
  SortBufs sb{};
  sb.tile_sums = tile_sums;
  sb.total = total;
  return scan_u32(in, out, n, sb, st);
}

int64_t scan_tile_count(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

psi_status build_schedule(const int* row_ptr, int64_t n, int64_t m, int items, int64_t n_tiles,
                          int* tile_row, hipStream_t st) {
  hipLaunchKernelGGL(k_schedule, dim3(grid_for(n_tiles + 1)), dim3(kBlock), 0, st, row_ptr, n, m,
                     int64_t(items), n_tiles, tile_row);
  PSI_HIP_CHECK(hipGetLastError());
  return PSI_OK;
}

}  // namespace psi
