// Random-gather probe: the access pattern of an operator pass without its
// arithmetic, to measure the ceiling the pass is held to.
//
// A pass over CSR(Aᵀ) streams one 4-byte column index per edge and gathers
// the 8-byte iterate entry it names; with S column segments the workgroups
// of XCD group s (blockIdx mod 8, mod S — XCDs receive workgroups
// round-robin) gather only inside segment s.  The probe does exactly that
// with the caller's indices: workgroup b sums x[s·seg + idx[k]] over its
// share of k, where s = (b mod 8) mod S, and writes the sum (so the loads
// cannot be dropped).  Gathers per second = n_idx / time.
#include <algorithm>

#include "psi_internal.h"

namespace psi {

namespace {

__global__ __launch_bounds__(kBlock) void k_gather_probe(const double* x, int64_t seg, int S,
                                                         const int* idx, int64_t n_idx,
                                                         double* out) {
  __shared__ double red[kBlock / 64];
  const int s = static_cast<int>(blockIdx.x & 7u) % S;
  const double* xs = x + int64_t(s) * seg;
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  // indices are clamped into the segment, so any input stays in bounds
  const uint32_t last = static_cast<uint32_t>(seg - 1);
  auto at = [&](int j) { return xs[min(static_cast<uint32_t>(j), last)]; };
  for (; k + 3 * stride < n_idx; k += 4 * stride) {
    const int j0 = idx[k], j1 = idx[k + stride], j2 = idx[k + 2 * stride], j3 = idx[k + 3 * stride];
    acc += (at(j0) + at(j1)) + (at(j2) + at(j3));
  }
  for (; k < n_idx; k += stride) acc += at(idx[k]);
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace

psi_status gather_probe(const double* x, int64_t n_x, int S, const int32_t* idx, int64_t n_idx,
                        double* out, int grid, int reps, double* mean_ms, hipStream_t st) {
  PSI_REQUIRE(x && idx && out && mean_ms, "pointers must not be NULL");
  PSI_REQUIRE(S == 1 || S == 2 || S == 4 || S == 8, "S must be 1, 2, 4 or 8");
  PSI_REQUIRE(n_x >= S && n_idx >= 1 && reps >= 1, "n_x >= S, n_idx >= 1 and reps >= 1 needed");
  PSI_REQUIRE(n_x / S <= (int64_t(1) << 31), "a segment must have at most 2^31 entries");
  PSI_REQUIRE(grid >= 8 && grid <= 65536 && grid % 8 == 0, "grid must be a multiple of 8 in [8, 65536]");
  const int64_t seg = n_x / S;
  hipLaunchKernelGGL(k_gather_probe, dim3(grid), dim3(kBlock), 0, st, x, seg, S, idx, n_idx, out);
  PSI_HIP_CHECK(hipGetLastError());
  EventPair evp;
  PSI_HIP_CHECK(hipEventCreate(&evp.a));
  PSI_HIP_CHECK(hipEventCreate(&evp.b));
  hipEvent_t a = evp.a, b = evp.b;
  PSI_HIP_CHECK(hipEventRecord(a, st));
  for (int r = 0; r < reps; ++r)
    hipLaunchKernelGGL(k_gather_probe, dim3(grid), dim3(kBlock), 0, st, x, seg, S, idx, n_idx,
                       out);
  PSI_HIP_CHECK(hipEventRecord(b, st));
  PSI_HIP_CHECK(hipEventSynchronize(b));
  float ms = 0.f;
  PSI_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
  PSI_HIP_CHECK(hipGetLastError());
  *mean_ms = static_cast<double>(ms) / reps;
  return PSI_OK;
}

}  // namespace psi
