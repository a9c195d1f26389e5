// Binned layout of CSR(Aᵀ) for the two-launch pass, built on first use.
//
// The pull sᵀA of eq. (power_psi) reads z_j = s_j/den_j at random followers
// j.  Past the caches (320 MB of FP64 z at 4·10⁷ users) each such read costs
// a cache line for 8 useful bytes.  The binned pass reorders the work so that
// every read of z comes from LDS and everything else streams (propagation
// blocking, Beamer, Asanović and Patterson, IPDPS 2017):
//   * followers are cut into column blocks of kBinsCols users (160 KB of
//     FP64 z, a CU's whole LDS); leaders into bins, row blocks of at most
//     kBinsRows rows and an edge budget, planned as the band layout's (a row
//     longer than the budget becomes pieces, each its own bin, added in order
//     afterwards);
//   * a run is the set of edges of one (column block, bin) pair, ordered by
//     (row, column);
//   * expand launch: one workgroup per column block loads the block's z into
//     LDS, then streams the block's entries (its runs, bins in order; each a
//     15-bit column within the block) and writes z of each entry to the
//     entry's slot in bin order: a run's slots are consecutive, so a run is
//     one contiguous write;
//   * bin launch: one wave per bin streams the bin's values and 16-bit rows
//     (its runs, column blocks in order) and adds them to its rows' sums in
//     LDS, then applies the epilogue.
// Every row's sum has a fixed order (column blocks in turn, followers
// ascending within each), so passes are bitwise repeatable.
//
// Tables: cnt[b][c] (edges of bin b in column block c); p2 = its exclusive
// scan in (bin, column block) order gives each run's first slot in bin order;
// p1 = the exclusive scan of the transposed counts in (column block, bin)
// order gives its first entry in expand order.  The non-empty runs, numbered
// in expand order, keep p2 − p1 (mod 2^32) in rdelta; an entry k of run r
// goes to slot rdelta[r] + k.  An expand wave knows its runs from the
// kBinsFirst flags of its entries, counted from the run before its first
// entry (task table).  The count tables live in the value array until the
// first pass overwrites it.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "psi_internal.h"

namespace psi {

namespace {

inline unsigned grid_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }
inline size_t round256(size_t x) { return (x + 255) / 256 * 256; }

// Edges of each bin per column block (one workgroup per bin, LDS histogram).
__global__ __launch_bounds__(kBlock) void k_bins_count(const int* col, const BandBlock* blocks,
                                                      int nb, int B, uint32_t* cnt) {
  extern __shared__ uint32_t hist[];
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < B; c += kBlock) hist[c] = 0u;
  __syncthreads();
  const int e_lo = blocks[b].e_lo, e_hi = blocks[b + 1].e_lo;
  for (int e = e_lo + static_cast<int>(threadIdx.x); e < e_hi; e += kBlock)
    atomicAdd(&hist[col[e] / kBinsCols], 1u);
  __syncthreads();
  for (int c = threadIdx.x; c < B; c += kBlock) cnt[int64_t(b) * B + c] = hist[c];
}

// out[c·rows_in + b] = in[b·cols_in + c], 64 x 64 tiles through LDS.
__global__ __launch_bounds__(kBlock) void k_transpose_u32(const uint32_t* in, uint32_t* out,
                                                         int64_t rows_in, int64_t cols_in) {
  __shared__ uint32_t t[64][65];
  const int64_t r0 = int64_t(blockIdx.y) * 64, c0 = int64_t(blockIdx.x) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += kBlock / 64) {
    const int64_t r = r0 + i, c = c0 + tx;
    t[i][tx] = r < rows_in && c < cols_in ? in[r * cols_in + c] : 0u;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += kBlock / 64) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols_in && r < rows_in) out[c * rows_in + r] = t[tx][i];
  }
}

// 1 where the count is non-zero.
__global__ __launch_bounds__(kBlock) void k_nonzero_u32(const uint32_t* in, uint32_t* out,
                                                       int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] = in[i] != 0u ? 1u : 0u;
}

// Per run (c, b) in expand order, from the counts in c-major order t (entry
// c·nb + b; ord = exclusive scan of the non-zero flags, so run (c, b) is
// non-empty iff ord[i + 1] > ord[i]): rdelta and the first entry p1 of the
// run (kept in rp1 for the task search).  Also per column block its first
// entry (cs) and first run (crun).
__global__ __launch_bounds__(kBlock) void k_bins_runs(const uint32_t* p1, const uint32_t* ord,
                                                     const uint32_t* p2, int nb, int B,
                                                     uint32_t* rdelta, uint32_t* rp1,
                                                     uint32_t* cs, uint32_t* crun, uint32_t m) {
  const int64_t n = int64_t(nb) * B;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int c = static_cast<int>(i / nb), b = static_cast<int>(i % nb);
  if (b == 0) {
    cs[c] = p1[i];
    crun[c] = ord[i];
    if (c == B - 1) {
      cs[B] = m;
      crun[B] = ord[n];
    }
  }
  if (ord[i + 1] > ord[i]) {
    const uint32_t r = ord[i];
    rdelta[r] = p2[int64_t(b) * B + c] - p1[i];
    rp1[r] = p1[i];
  }
}

// Per (column block, expand wave): the run before the wave's first entry, so
// that counting the kBinsFirst flags from there gives every entry's run.
__global__ __launch_bounds__(kBlock) void k_bins_tasks(const uint32_t* cs, const uint32_t* crun,
                                                      const uint32_t* rp1, int B, int* task) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= B * kBinsExpandWaves) return;
  const int c = i / kBinsExpandWaves, w = i % kBinsExpandWaves;
  const uint32_t lo0 = cs[c], ne = cs[c + 1] - cs[c];
  const uint32_t lo = lo0 + static_cast<uint32_t>((uint64_t(ne) * w) / kBinsExpandWaves);
  const uint32_t hi = lo0 + static_cast<uint32_t>((uint64_t(ne) * (w + 1)) / kBinsExpandWaves);
  int r0 = static_cast<int>(crun[c]), r1 = static_cast<int>(crun[c + 1]);
  if (lo >= hi || r0 >= r1) {
    task[i] = r0;
    return;
  }
  // the last run of the column block starting at or before lo
  int a = r0, z = r1 - 1;
  while (a < z) {
    const int mid = (a + z + 1) >> 1;
    if (rp1[mid] <= lo) a = mid; else z = mid - 1;
  }
  task[i] = rp1[a] == lo ? a - 1 : a;
}

// First bin-order entry of each bin: p2 at (b, 0).
__global__ __launch_bounds__(kBlock) void k_bins_bstart(const uint32_t* p2, int nb, int B,
                                                       uint32_t m, uint32_t* bstart) {
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b < nb) bstart[b] = p2[int64_t(b) * B];
  if (b == nb) bstart[nb] = m;
}

// The entries (one wave per bin): the bin's edges in CSR order, each ranked
// within its run by a cursor per column block in LDS (lanes of one chunk with
// the same column block ranked by ballots over the block index bits); its row
// goes to slot p2 + rank in bin order, its column to entry p1 + rank in
// expand order, the run's first entry flagged in both.
__global__ __launch_bounds__(64) void k_bins_fill(const int* row_ptr, const int* col,
                                                 const BandBlock* blocks, int nb, int B,
                                                 int cbits, const uint32_t* p2,
                                                 const uint32_t* p1, uint16_t* rows16,
                                                 uint16_t* cols16) {
  extern __shared__ uint32_t cur[];
  const int lane = threadIdx.x;
  const int b = blockIdx.x;
  for (int c = lane; c < B; c += 64) cur[c] = 0u;
  __builtin_amdgcn_wave_barrier();
  const BandBlock bb = blocks[b];
  const int e_hi = blocks[b + 1].e_lo;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int e0 = bb.e_lo; e0 < e_hi; e0 += 64) {
    const int e = e0 + lane;
    const bool valid = e < e_hi;
    int j = 0, rl = 0;
    if (valid) {
      j = col[e];
      int lo = 0, hi = bb.nrows - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_ptr[bb.row_lo + mid] <= e) lo = mid; else hi = mid - 1;
      }
      rl = lo;
    }
    const int c = valid ? (j / kBinsCols) : 0;
    unsigned long long peers = __ballot(valid);
    for (int bit = 0; bit < cbits; ++bit) {
      const bool one = (c >> bit) & 1;
      const unsigned long long m1 = __ballot(one);
      peers &= one ? m1 : ~m1;
    }
    const uint32_t base = valid ? cur[c] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      const uint32_t rank = base + static_cast<uint32_t>(__popcll(peers & below));
      const uint16_t first = rank == 0u ? static_cast<uint16_t>(kBinsFirst) : uint16_t(0);
      rows16[p2[int64_t(b) * B + c] + rank] = static_cast<uint16_t>(rl) | first;
      cols16[p1[int64_t(c) * nb + b] + rank] =
          static_cast<uint16_t>(j - c * kBinsCols) | first;
      if ((peers >> lane) == 1ull) cur[c] = base + static_cast<uint32_t>(__popcll(peers));
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Greedy bin plan (rows in order, at most `rows` rows and emax edges a bin; a
// longer row becomes pieces), as the band layout's.
void plan_bins(const std::vector<int>& rp, int64_t n, int rows, int64_t emax,
               std::vector<BandBlock>& blocks, std::vector<int4>& split) {
  blocks.clear();
  split.clear();
  int piece = 0;
  int64_t i = 0;
  while (i < n) {
    const int64_t len = int64_t(rp[i + 1]) - rp[i];
    if (len > emax) {
      const int64_t k = (len + emax - 1) / emax;
      const int p0 = piece;
      for (int64_t q = 0; q < k; ++q) {
        const int64_t lo = rp[i] + len * q / k;
        blocks.push_back(BandBlock{static_cast<int>(i), 1, piece++, static_cast<int>(lo)});
      }
      split.push_back(int4{static_cast<int>(i), p0, piece,
                           static_cast<int>(blocks.size()) - 1});
      ++i;
      continue;
    }
    int64_t j = i, edges = 0;
    while (j < n && j - i < rows) {
      const int64_t l = int64_t(rp[j + 1]) - rp[j];
      if (l > emax || (j > i && edges + l > emax)) break;
      edges += l;
      ++j;
    }
    blocks.push_back(BandBlock{static_cast<int>(i), static_cast<int>(j - i), -1, rp[i]});
    i = j;
  }
}

}  // namespace

psi_status ensure_bins(psi_operator* op, hipStream_t st) {
  PSI_REQUIRE(op->n_graphs == 1, "the binned layout is for single-graph operators");
  PSI_REQUIRE(op->bins_val != nullptr, "the binned layout has no workspace");
  if (op->bins_built) return PSI_OK;
  const int64_t n = op->n;
  const int64_t m = op->m;
  PSI_REQUIRE(m < (int64_t(1) << 32) - 1, "too many edges for the binned layout");
  const int64_t B = (n + kBinsCols - 1) / kBinsCols;
  PSI_REQUIRE(B >= 1 && B <= kBinsMaxB && B <= op->cap_bins_cols,
              "too many column blocks for the binned layout");
  std::vector<int> rp(n + 1);
  PSI_HIP_CHECK(hipMemcpyAsync(rp.data(), op->row_ptr, 4 * size_t(n + 1), hipMemcpyDeviceToHost,
                               st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  // edge budget at least 2.5·R·M/N: then the plan has at most 3·ceil(N/R) + 1
  // bins (rows closed by count, by budget, before a split row, pieces), which
  // the workspace reserves
  const double per_row = n > 0 ? static_cast<double>(m) / static_cast<double>(n) : 0.0;
  const int64_t emax = std::max<int64_t>(
      kBinsMinEdges, static_cast<int64_t>(std::ceil(2.5 * kBinsRows * per_row)));
  std::vector<BandBlock> blocks;
  std::vector<int4> split;
  plan_bins(rp, n, kBinsRows, emax, blocks, split);
  const int64_t nb = static_cast<int64_t>(blocks.size());
  PSI_REQUIRE(nb >= 1 && nb <= op->cap_bins_blocks, "the bin plan exceeds its reserved capacity");
  blocks.push_back(BandBlock{static_cast<int>(n), 0, -1, static_cast<int>(m)});  // sentinel
  // launch order: most edges first, so that the longest bins do not end the launch
  std::vector<int> order(nb);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    return blocks[x + 1].e_lo - blocks[x].e_lo > blocks[y + 1].e_lo - blocks[y].e_lo;
  });
  // count tables in the value array: cnt → p2 (in place), its transpose → p1
  // (in place), the non-empty flags' scan → ord, and the scans' tile sums
  const int64_t nt = nb * B;
  const size_t tab = round256(4 * size_t(nt + 1));
  const size_t tiles = round256(4 * size_t(scan_tile_count(nt + 1) + 2));
  PSI_REQUIRE(3 * tab + tiles + round256(4 * size_t(nt + 1)) <= op->cap_bins_val || m == 0,
              "the binned layout's count tables do not fit its value array");
  PSI_REQUIRE(std::min<int64_t>(nt, m) <= op->cap_bins_runs, "the bin runs exceed their capacity");
  PSI_HIP_CHECK(hipMemcpyAsync(op->bins_blocks, blocks.data(), sizeof(BandBlock) * blocks.size(),
                               hipMemcpyHostToDevice, st));
  if (!split.empty())
    PSI_HIP_CHECK(hipMemcpyAsync(op->bins_split, split.data(), sizeof(int4) * split.size(),
                                 hipMemcpyHostToDevice, st));
  PSI_HIP_CHECK(hipMemcpyAsync(op->bins_order, order.data(), sizeof(int) * order.size(),
                               hipMemcpyHostToDevice, st));
  if (m > 0) {
    char* base = static_cast<char*>(op->bins_val);
    uint32_t* cnt = reinterpret_cast<uint32_t*>(base);            // → p2
    uint32_t* cntT = reinterpret_cast<uint32_t*>(base + tab);     // → p1
    uint32_t* ord = reinterpret_cast<uint32_t*>(base + 2 * tab);
    uint32_t* tsum = reinterpret_cast<uint32_t*>(base + 3 * tab);
    uint32_t* rp1 = reinterpret_cast<uint32_t*>(base + 3 * tab + tiles);
    uint32_t* total = tsum + scan_tile_count(nt + 1) + 1;
    hipLaunchKernelGGL(k_bins_count, dim3(unsigned(nb)), dim3(kBlock), 4 * size_t(B), st, op->col,
                       op->bins_blocks, static_cast<int>(nb), static_cast<int>(B), cnt);
    PSI_HIP_CHECK(hipMemsetAsync(cnt + nt, 0, 4, st));
    hipLaunchKernelGGL(k_transpose_u32, dim3(unsigned((B + 63) / 64), unsigned((nb + 63) / 64)),
                       dim3(kBlock), 0, st, cnt, cntT, nb, B);
    PSI_HIP_CHECK(hipMemsetAsync(cntT + nt, 0, 4, st));
    hipLaunchKernelGGL(k_nonzero_u32, dim3(grid_for(nt + 1)), dim3(kBlock), 0, st, cntT, ord,
                       nt + 1);
    uint32_t sums[3] = {0u, 0u, 0u};
    psi_status s = scan_exclusive_u32(cnt, cnt, nt + 1, tsum, total, st);
    if (s != PSI_OK) return s;
    PSI_HIP_CHECK(hipMemcpyAsync(&sums[0], total, 4, hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    s = scan_exclusive_u32(cntT, cntT, nt + 1, tsum, total, st);
    if (s != PSI_OK) return s;
    PSI_HIP_CHECK(hipMemcpyAsync(&sums[1], total, 4, hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    s = scan_exclusive_u32(ord, ord, nt + 1, tsum, total, st);
    if (s != PSI_OK) return s;
    PSI_HIP_CHECK(hipMemcpyAsync(&sums[2], total, 4, hipMemcpyDeviceToHost, st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    if (int64_t(sums[0]) != m || int64_t(sums[1]) != m) {
      set_error("the binned layout lost edges");
      return PSI_EDEVICE;
    }
    const int64_t runs = sums[2];
    PSI_REQUIRE(runs <= op->cap_bins_runs, "the bin runs exceed their capacity");
    hipLaunchKernelGGL(k_bins_runs, dim3(grid_for(nt)), dim3(kBlock), 0, st, cntT, ord, cnt,
                       static_cast<int>(nb), static_cast<int>(B), op->bins_rdelta, rp1,
                       op->bins_cs, op->bins_crun, static_cast<uint32_t>(m));
    hipLaunchKernelGGL(k_bins_tasks, dim3(grid_for(B * kBinsExpandWaves)), dim3(kBlock), 0, st,
                       op->bins_cs, op->bins_crun, rp1, static_cast<int>(B), op->bins_task);
    hipLaunchKernelGGL(k_bins_bstart, dim3(grid_for(nb + 1)), dim3(kBlock), 0, st, cnt,
                       static_cast<int>(nb), static_cast<int>(B), static_cast<uint32_t>(m),
                       op->bins_bstart);
    int cbits = 0;
    while ((int64_t(1) << cbits) < B) ++cbits;
    hipLaunchKernelGGL(k_bins_fill, dim3(unsigned(nb)), dim3(64), 4 * size_t(B), st, op->row_ptr,
                       op->col, op->bins_blocks, static_cast<int>(nb), static_cast<int>(B), cbits,
                       cnt, cntT, op->bins_row, op->bins_col);
    PSI_HIP_CHECK(hipGetLastError());
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    op->bins_runs = runs;
  } else {
    std::vector<uint32_t> zeros(size_t(nb + 1), 0u);
    PSI_HIP_CHECK(hipMemcpyAsync(op->bins_bstart, zeros.data(), 4 * size_t(nb + 1),
                                 hipMemcpyHostToDevice, st));
    std::vector<uint32_t> zb(size_t(B + 1), 0u);
    PSI_HIP_CHECK(hipMemcpyAsync(op->bins_cs, zb.data(), 4 * size_t(B + 1), hipMemcpyHostToDevice,
                                 st));
    PSI_HIP_CHECK(hipMemcpyAsync(op->bins_crun, zb.data(), 4 * size_t(B + 1),
                                 hipMemcpyHostToDevice, st));
    std::vector<int> zt(size_t(B) * kBinsExpandWaves, 0);
    PSI_HIP_CHECK(hipMemcpyAsync(op->bins_task, zt.data(), 4 * zt.size(), hipMemcpyHostToDevice,
                                 st));
    PSI_HIP_CHECK(hipStreamSynchronize(st));
    op->bins_runs = 0;
  }
  op->bins_B = static_cast<int>(B);
  op->bins_nb = static_cast<int>(nb);
  op->bins_n_split = static_cast<int>(split.size());
  op->bins_built = true;
  return PSI_OK;
}

}  // namespace psi
