// Column-blocked ("band") layout of CSR(Aᵀ), built on first use.
//
// The pull sᵀA of eq. (power_psi) gathers z_j = s_j/den_j at random followers
// j.  When z exceeds what the caches hold (320 MB in FP64 at 4·10⁷ users,
// beyond the 256 MB Infinity Cache and far beyond an XCD's 4 MB L2), every
// gather costs a line from HBM.  The band layout makes the gathers hit L2:
//   * columns (followers) are cut into blocks of W = 2^wlog users, 1-2 MB of
//     z, which an XCD's L2 keeps;
//   * rows (leaders) are cut into row blocks, each of at most R rows and about
//     E edges, summed by one wave that keeps its rows' sums in LDS; a row
//     longer than E is cut into pieces, each its own row block, whose sums a
//     small kernel adds in order afterwards;
//   * a launch runs one row block per wave for as many waves as the device
//     holds at once (a "band"), and every wave walks its row block's edges
//     column block by column block, so all waves of a launch gather from the
//     same 1-2 MB of z at about the same time; bands run one after another.
// A row block's entries are its edges ordered by (column block, row, column):
// 32 bits each, (row within the block) << wlog | (column within the block).
// The entries of row block b in column block c are
// [toff[b·B + c], toff[b·B + c + 1]).  Every row's sum therefore has a fixed
// order (column blocks in turn, followers ascending within each), so passes
// are bitwise repeatable.
//
// Build: the row-block plan is made on the host from row_ptr (greedy, rows in
// order); one wave per row block counts its entries per column block; an
// exclusive scan gives toff; one wave per row block then writes its entries,
// edges in CSR order, each to its column block's next slot (lanes with the
// same column block ranked by ballots over the block index bits).
#include <algorithm>
#include <cmath>
#include <vector>

#include "psi_internal.h"

namespace psi {

namespace {

inline unsigned grid_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

// Entries of each row block per column block (one wave per row block).
__global__ __launch_bounds__(kBlock) void k_band_count(const int* col, const BandBlock* blocks,
                                                      int n_blocks, int B, int wlog,
                                                      uint32_t* cnt) {
  __shared__ uint32_t hist[kBlock / 64][kBandMaxCols];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.x * (kBlock / 64) + wave;
  if (b >= n_blocks) return;  // waves are independent: no barrier below
  uint32_t* h = hist[wave];
  for (int c = lane; c < B; c += 64) h[c] = 0u;
  __builtin_amdgcn_wave_barrier();
  const int e_lo = blocks[b].e_lo, e_hi = blocks[b + 1].e_lo;
  for (int e = e_lo + lane; e < e_hi; e += 64) atomicAdd(&h[col[e] >> wlog], 1u);
  __builtin_amdgcn_wave_barrier();
  for (int c = lane; c < B; c += 64) cnt[int64_t(b) * B + c] = h[c];
}

// The entries of each row block (one wave per row block): its edges in CSR
// order, each to the next slot of its column block.
__global__ __launch_bounds__(kBlock) void k_band_fill(const int* row_ptr, const int* col,
                                                     const BandBlock* blocks, int n_blocks, int B,
                                                     int wlog, int cbits, const uint32_t* toff,
                                                     uint32_t* ent) {
  __shared__ uint32_t cur[kBlock / 64][kBandMaxCols];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int b = blockIdx.x * (kBlock / 64) + wave;
  if (b >= n_blocks) return;
  uint32_t* cu = cur[wave];
  for (int c = lane; c < B; c += 64) cu[c] = toff[int64_t(b) * B + c];
  __builtin_amdgcn_wave_barrier();
  const BandBlock bb = blocks[b];
  const int e_hi = blocks[b + 1].e_lo;
  const uint32_t wmask = (1u << wlog) - 1u;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int e0 = bb.e_lo; e0 < e_hi; e0 += 64) {
    const int e = e0 + lane;
    const bool valid = e < e_hi;
    int j = 0, rl = 0;
    if (valid) {
      j = col[e];
      // the row holding edge e: the last row r of the block with row_ptr[r] <= e
      int lo = 0, hi = bb.nrows - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_ptr[bb.row_lo + mid] <= e) lo = mid; else hi = mid - 1;
      }
      rl = lo;
    }
    const int c = valid ? (j >> wlog) : 0;
    // lanes whose edge goes to the same column block, by ballots over its bits
    unsigned long long peers = __ballot(valid);
    for (int bit = 0; bit < cbits; ++bit) {
      const bool one = (c >> bit) & 1;
      const unsigned long long m1 = __ballot(one);
      peers &= one ? m1 : ~m1;
    }
    const uint32_t base = valid ? cu[c] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      const uint32_t pos = base + static_cast<uint32_t>(__popcll(peers & below));
      ent[pos] = (static_cast<uint32_t>(rl) << wlog) | (static_cast<uint32_t>(j) & wmask);
      // the highest lane of the group advances its column block's cursor
      if ((peers >> lane) == 1ull) cu[c] = base + static_cast<uint32_t>(__popcll(peers));
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Greedy row-block plan: rows in order into blocks of at most `rows` rows and
// `emax` edges; a row longer than emax becomes pieces of at most emax edges,
// one block each.
void plan_blocks(const std::vector<int>& rp, int64_t n, int rows, int64_t emax,
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

int band_waves(int rows);

// Build (or keep) the band layout for column blocks of 2^wlog users and row
// blocks of at most `rows` rows.
psi_status ensure_bands(psi_operator* op, int wlog, int rows, hipStream_t st) {
  PSI_REQUIRE(wlog >= kBandMinLog && wlog <= kBandMaxLog, "unsupported band column width");
  PSI_REQUIRE(band_rows_supported(rows), "unsupported band row-block size");
  PSI_REQUIRE(op->n_graphs == 1, "the band layout is for single-graph operators");
  if (op->band_built && op->band_wlog == wlog && op->band_rows == rows) return PSI_OK;
  op->band_built = false;
  const int64_t n = op->n;
  const int64_t m = op->m;
  const int64_t B = (n + (int64_t(1) << wlog) - 1) >> wlog;
  PSI_REQUIRE(B >= 1 && B <= kBandMaxCols && B <= op->cap_band_cols,
              "too many column blocks for the band layout");
  const int waves = band_waves(rows);
  if (waves <= 0) {
    set_error("could not size the band launch");
    return PSI_EDEVICE;
  }
  std::vector<int> rp(n + 1);
  PSI_HIP_CHECK(hipMemcpyAsync(rp.data(), op->row_ptr, 4 * size_t(n + 1), hipMemcpyDeviceToHost,
                               st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  // bands: enough that every row block fits `rows` rows; edges per block
  // sized so that the blocks of those bands carry the edges with 10% slack
  const int64_t by_rows = (n + int64_t(waves) * rows - 1) / (int64_t(waves) * rows);
  const int64_t k = std::max<int64_t>(1, by_rows);
  int64_t emax = std::max<int64_t>(kBandMinEdges, (m * 11 / 10 + k * waves - 1) / (k * waves));
  std::vector<BandBlock> blocks;
  std::vector<int4> split;
  plan_blocks(rp, n, rows, emax, blocks, split);
  const int64_t nb = static_cast<int64_t>(blocks.size());
  PSI_REQUIRE(nb + 1 <= op->cap_band_blocks, "the band plan exceeds its reserved capacity");
  PSI_REQUIRE(nb * B + 1 <= op->cap_band_toff, "the band offsets exceed their reserved capacity");
  blocks.push_back(BandBlock{static_cast<int>(n), 0, -1, static_cast<int>(m)});  // sentinel
  PSI_HIP_CHECK(hipMemcpyAsync(op->band_blocks, blocks.data(), sizeof(BandBlock) * blocks.size(),
                               hipMemcpyHostToDevice, st));
  if (!split.empty())
    PSI_HIP_CHECK(hipMemcpyAsync(op->band_split, split.data(), sizeof(int4) * split.size(),
                                 hipMemcpyHostToDevice, st));
  const unsigned grid = static_cast<unsigned>((nb + kBlock / 64 - 1) / (kBlock / 64));
  if (m > 0) {
    hipLaunchKernelGGL(k_band_count, dim3(grid), dim3(kBlock), 0, st, op->col, op->band_blocks,
                       static_cast<int>(nb), static_cast<int>(B), wlog, op->band_toff);
  } else {
    PSI_HIP_CHECK(hipMemsetAsync(op->band_toff, 0, 4 * size_t(nb * B), st));
  }
  PSI_HIP_CHECK(hipMemsetAsync(op->band_toff + nb * B, 0, 4, st));
  uint32_t total = 0;
  psi_status s = scan_exclusive_u32(op->band_toff, op->band_toff, nb * B + 1, op->band_scan_tmp,
                                    op->band_scan_tmp + scan_tile_count(nb * B + 1) + 1, st);
  if (s != PSI_OK) return s;
  PSI_HIP_CHECK(hipMemcpyAsync(&total, op->band_toff + nb * B, 4, hipMemcpyDeviceToHost, st));
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  if (int64_t(total) != m) {
    set_error("the band layout lost edges");
    return PSI_EDEVICE;
  }
  int cbits = 0;
  while ((int64_t(1) << cbits) < B) ++cbits;
  if (m > 0)
    hipLaunchKernelGGL(k_band_fill, dim3(grid), dim3(kBlock), 0, st, op->row_ptr, op->col,
                       op->band_blocks, static_cast<int>(nb), static_cast<int>(B), wlog, cbits,
                       op->band_toff, op->band_ent);
  PSI_HIP_CHECK(hipGetLastError());
  PSI_HIP_CHECK(hipStreamSynchronize(st));
  op->band_wlog = wlog;
  op->band_rows = rows;
  op->band_B = static_cast<int>(B);
  op->band_nb = static_cast<int>(nb);
  op->band_waves = waves;
  op->band_count = static_cast<int>((nb + waves - 1) / waves);
  op->band_n_split = static_cast<int>(split.size());
  // per band: its first row, and the split rows whose pieces all lie in it or
  // an earlier band (a Gauss–Seidel sweep finishes them after that band)
  op->band_row0.assign(op->band_count + 1, static_cast<int>(n));
  op->band_split_end.assign(op->band_count, 0);
  for (int k = 0; k < op->band_count; ++k) {
    op->band_row0[k] = blocks[size_t(k) * waves].row_lo;
    const int64_t end_block = std::min<int64_t>(nb, int64_t(k + 1) * waves);
    int q = k ? op->band_split_end[k - 1] : 0;
    while (q < static_cast<int>(split.size()) && split[q].w < end_block) ++q;
    op->band_split_end[k] = q;
  }
  op->band_built = true;
  return PSI_OK;
}

}  // namespace psi
